// api.cpp -- the C ABI: argument checks, plan construction, launch
// configuration, autotuning and HIP-graph capture.  Hot-path entry points only
// check arguments on the host and enqueue kernels.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/zfpx.h"
#include "internal.hpp"

using namespace zfpx;

namespace {

constexpr int64_t kMaxBlocks = kMaxPlanBlocks;

bool rate_ok(int rate) { return rate >= 1 && rate <= 32; }
int64_t ceil4(int64_t n) { return (n + 3) / 4; }
bool aligned(const void* p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

// One tile per wavefront.  Two wavefronts per workgroup for launches up to
// 2^16 tiles (timed on the z->lambda share, 14,105 tiles, encode and decode
// alternating: 64 threads lose 5% and 256 match), one above (on the 9.47 GB
// buffer, 591,560 tiles, 64 threads are 1-2% faster than 128 at rates 8 and
// 16, both ops, and 256 slower).
constexpr int64_t kManyTilesBlocks = int64_t(64) << 16;
LaunchCfg default_cfg(int, int64_t nblocks) {
  LaunchCfg c;
  c.wg = nblocks > kManyTilesBlocks ? 64 : 128;
  c.grid = 0;
  return c;
}

bool cfg_ok(LaunchCfg c, int rate) {
  if (c.wg != 64 && c.wg != 128 && c.wg != 256) return false;
  if (c.grid < 0) return false;
  return lds_bytes(c.wg, rate) <= device_max_lds();
}

}  // namespace

struct zfpx_plan {
  int32_t nchunks = 0;
  int64_t nblocks = 0, nvalues = 0, min_elems = 0;
  bool vec4 = true;
  std::vector<int64_t> chunk_blocks, chunk_first;  // host copies
  std::vector<int64_t> shape_key;                   // for the tuning cache
  SegDesc* d_segs = nullptr;
  int32_t* d_seg_block0 = nullptr;
  int32_t* d_tile_seg = nullptr;
  int64_t* d_chunk_first = nullptr;  // [nchunks + 1], for the variable-size chunk offsets
  PlanDev dev{};
  std::map<std::pair<int, int>, LaunchCfg> cfg;  // (op, rate) -> config; rate 0 = any

  LaunchCfg config(int op, int rate) const {
    auto it = cfg.find({op, rate});
    if (it != cfg.end()) return it->second;
    it = cfg.find({op, 0});
    if (it != cfg.end() && lds_bytes(it->second.wg, rate) <= device_max_lds()) return it->second;
    return default_cfg(op, nblocks);
  }
};

struct zfpx_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

const char* zfpx_status_string(int status) {
  switch (status) {
    case ZFPX_OK: return "ok";
    case ZFPX_EINVAL: return "invalid argument";
    case ZFPX_ENOSPC: return "output buffer too small";
    case ZFPX_EHIP: return "HIP runtime error";
    case ZFPX_ENOMEM: return "out of memory";
    case ZFPX_EAGAIN: return "queue full, try again";
    case ZFPX_ESTATE: return "invalid state";
    default: return "unknown status";
  }
}

int zfpx_version(void) { return 100; }

int zfpx_device_cus(void) { return device_cu_count(); }

int64_t zfpx_fixed_rate_bytes(int64_t nx, int64_t ny, int64_t nz, int rate) {
  if (!rate_ok(rate) || nx < 0 || ny < 0 || nz < 0) return ZFPX_EINVAL;
  int64_t nb = ceil4(nx) * ceil4(ny) * ceil4(nz);
  return nb * 8 * rate;
}

// ---------------------------------------------------------------------------
// Regular arrays
// ---------------------------------------------------------------------------

static int regular_setup(int64_t nx, int64_t ny, int64_t nz, int64_t sx, int64_t sy, int64_t sz,
                         int rate, RegularDev* g, int64_t* nblocks) {
  if (!rate_ok(rate) || nx < 0 || ny < 0 || nz < 0) return ZFPX_EINVAL;
  int64_t nbx = ceil4(nx), nby = ceil4(ny), nbz = ceil4(nz);
  int64_t nb = nbx * nby * nbz;
  if (nb > kMaxBlocks) return ZFPX_EINVAL;
  *g = RegularDev{nx, ny, nz, sx, sy, sz, (int32_t)nbx, (int32_t)nby};
  *nblocks = nb;
  return ZFPX_OK;
}

static bool regular_vec4(const void* p, int64_t sx, int64_t sy, int64_t sz) {
  return sx == 1 && (sy & 3) == 0 && (sz & 3) == 0 && aligned(p, 16);
}

int zfpx_encode_fixed_rate(const float* d_in, int64_t nx, int64_t ny, int64_t nz, int64_t sx,
                           int64_t sy, int64_t sz, int rate, void* d_out, size_t out_bytes,
                           void* stream) {
  RegularDev g;
  int64_t nb;
  int st = regular_setup(nx, ny, nz, sx, sy, sz, rate, &g, &nb);
  if (st) return st;
  if (nb == 0) return ZFPX_OK;
  if (!d_in || !d_out || !aligned(d_out, 8)) return ZFPX_EINVAL;
  if ((int64_t)out_bytes < nb * 8 * rate) return ZFPX_ENOSPC;
  hipError_t e = launch_regular_encode(g, regular_vec4(d_in, sx, sy, sz), d_in, (uint64_t*)d_out,
                                       rate, (int32_t)nb, default_cfg(kOpEncode, nb),
                                       (hipStream_t)stream);
  return e == hipSuccess ? ZFPX_OK : ZFPX_EHIP;
}

int zfpx_decode_fixed_rate(const void* d_in, size_t in_bytes, int64_t nx, int64_t ny, int64_t nz,
                           int64_t sx, int64_t sy, int64_t sz, int rate, float* d_out,
                           void* stream) {
  RegularDev g;
  int64_t nb;
  int st = regular_setup(nx, ny, nz, sx, sy, sz, rate, &g, &nb);
  if (st) return st;
  if (nb == 0) return ZFPX_OK;
  if (!d_in || !d_out || !aligned(d_in, 8)) return ZFPX_EINVAL;
  if ((int64_t)in_bytes < nb * 8 * rate) return ZFPX_ENOSPC;
  hipError_t e = launch_regular_decode(g, regular_vec4(d_out, sx, sy, sz), (const uint64_t*)d_in,
                                       d_out, rate, (int32_t)nb, default_cfg(kOpDecode, nb),
                                       (hipStream_t)stream);
  return e == hipSuccess ? ZFPX_OK : ZFPX_EHIP;
}

// ---------------------------------------------------------------------------
// Plans
// ---------------------------------------------------------------------------

int zfpx_plan_destroy(zfpx_plan* p) {
  if (!p) return ZFPX_EINVAL;
  if (p->d_segs) (void)hipFree(p->d_segs);
  if (p->d_seg_block0) (void)hipFree(p->d_seg_block0);
  if (p->d_tile_seg) (void)hipFree(p->d_tile_seg);
  if (p->d_chunk_first) (void)hipFree(p->d_chunk_first);
  delete p;
  return ZFPX_OK;
}

int zfpx_plan_create(int32_t nchunks, const int64_t* chunk_base, const int64_t* level_stride,
                     const int32_t* levels, const int32_t* row_start, const int64_t* row_offset,
                     const int32_t* row_len, zfpx_plan** out) {
  if (!out) return ZFPX_EINVAL;
  *out = nullptr;
  PlanTables t;
  if (build_plan_tables(nchunks, chunk_base, level_stride, levels, row_start, row_offset, row_len,
                        &t) != 0)
    return ZFPX_EINVAL;
  zfpx_plan* p = new (std::nothrow) zfpx_plan();
  if (!p) return ZFPX_ENOMEM;
  p->nchunks = nchunks;
  p->chunk_blocks = t.chunk_blocks;
  p->chunk_first = t.chunk_first;
  p->nblocks = t.nblocks;
  p->nvalues = t.nvalues;
  p->min_elems = t.min_elems;
  p->vec4 = t.vec4;
  p->shape_key = {nchunks, t.nblocks, t.nvalues, (int64_t)t.segs.size()};
  const std::vector<SegDesc>& segs = t.segs;
  if (!segs.empty()) {
    const size_t nseg = segs.size();
    if (hipMalloc(&p->d_segs, nseg * sizeof(SegDesc)) != hipSuccess ||
        hipMalloc(&p->d_seg_block0, (nseg + 1) * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&p->d_tile_seg, t.tile_seg.size() * sizeof(int32_t)) != hipSuccess) {
      zfpx_plan_destroy(p);
      return ZFPX_ENOMEM;
    }
    if (hipMemcpy(p->d_segs, segs.data(), nseg * sizeof(SegDesc), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(p->d_seg_block0, t.seg_block0.data(), (nseg + 1) * sizeof(int32_t),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_tile_seg, t.tile_seg.data(), t.tile_seg.size() * sizeof(int32_t),
                  hipMemcpyHostToDevice) != hipSuccess) {
      zfpx_plan_destroy(p);
      return ZFPX_EHIP;
    }
  }
  if (t.nblocks > 0) {
    if (hipMalloc(&p->d_chunk_first, ((size_t)nchunks + 1) * sizeof(int64_t)) != hipSuccess) {
      zfpx_plan_destroy(p);
      return ZFPX_ENOMEM;
    }
    if (hipMemcpy(p->d_chunk_first, p->chunk_first.data(), ((size_t)nchunks + 1) * sizeof(int64_t),
                  hipMemcpyHostToDevice) != hipSuccess) {
      zfpx_plan_destroy(p);
      return ZFPX_EHIP;
    }
  }
  p->dev = PlanDev{p->d_segs, p->d_seg_block0, p->d_tile_seg};
  (void)device_cu_count();  // device facts are queried here, outside any capture
  *out = p;
  return ZFPX_OK;
}

int zfpx_plan_info(const zfpx_plan* p, int64_t* nblocks, int64_t* nvalues,
                   int64_t* min_buffer_elems) {
  if (!p) return ZFPX_EINVAL;
  if (nblocks) *nblocks = p->nblocks;
  if (nvalues) *nvalues = p->nvalues;
  if (min_buffer_elems) *min_buffer_elems = p->min_elems;
  return ZFPX_OK;
}

int zfpx_plan_sizes(const zfpx_plan* p, int rate, int64_t* chunk_bytes, int64_t* chunk_offsets,
                    int64_t* total_bytes) {
  if (!p || !rate_ok(rate)) return ZFPX_EINVAL;
  for (int c = 0; c < p->nchunks; c++) {
    if (chunk_bytes) chunk_bytes[c] = p->chunk_blocks[c] * 8 * rate;
    if (chunk_offsets) chunk_offsets[c] = p->chunk_first[c] * 8 * rate;
  }
  if (total_bytes) *total_bytes = p->nblocks * 8 * rate;
  return ZFPX_OK;
}

static int plan_range(const zfpx_plan* p, int32_t first, int32_t count, int32_t* b0,
                      int32_t* b1) {
  if (first < 0 || count < 0 || (int64_t)first + count > p->nchunks) return ZFPX_EINVAL;
  *b0 = (int32_t)p->chunk_first[first];
  *b1 = (int32_t)p->chunk_first[first + count];
  return ZFPX_OK;
}

static int do_pack_encode(const zfpx_plan* p, int32_t first, int32_t count, const float* d_src,
                          int64_t src_elems, int rate, void* d_send, size_t send_bytes,
                          void* stream) {
  if (!p || !rate_ok(rate)) return ZFPX_EINVAL;
  int32_t b0, b1;
  int st = plan_range(p, first, count, &b0, &b1);
  if (st) return st;
  if (b1 == b0) return ZFPX_OK;
  if (!d_src || !d_send || !aligned(d_send, 8) || src_elems < p->min_elems) return ZFPX_EINVAL;
  if ((int64_t)send_bytes < p->nblocks * 8 * rate) return ZFPX_ENOSPC;
  bool vec4 = p->vec4 && aligned(d_src, 16);
  hipError_t e = launch_plan_encode(p->dev, vec4, d_src, (uint64_t*)d_send, rate, b0, b1,
                                    p->config(kOpEncode, rate), (hipStream_t)stream);
  return e == hipSuccess ? ZFPX_OK : ZFPX_EHIP;
}

static int do_decode_unpack(const zfpx_plan* p, int32_t first, int32_t count, const void* d_recv,
                            size_t recv_bytes, int rate, float* d_dst, int64_t dst_elems,
                            void* stream) {
  if (!p || !rate_ok(rate)) return ZFPX_EINVAL;
  int32_t b0, b1;
  int st = plan_range(p, first, count, &b0, &b1);
  if (st) return st;
  if (b1 == b0) return ZFPX_OK;
  if (!d_recv || !d_dst || !aligned(d_recv, 8) || dst_elems < p->min_elems) return ZFPX_EINVAL;
  if ((int64_t)recv_bytes < p->nblocks * 8 * rate) return ZFPX_ENOSPC;
  bool vec4 = p->vec4 && aligned(d_dst, 16);
  hipError_t e = launch_plan_decode(p->dev, vec4, (const uint64_t*)d_recv, d_dst, rate, b0, b1,
                                    p->config(kOpDecode, rate), (hipStream_t)stream);
  return e == hipSuccess ? ZFPX_OK : ZFPX_EHIP;
}

int zfpx_pack_encode(const zfpx_plan* p, const float* d_src, int64_t src_elems, int rate,
                     void* d_send, size_t send_bytes, void* stream) {
  if (!p) return ZFPX_EINVAL;
  return do_pack_encode(p, 0, p->nchunks, d_src, src_elems, rate, d_send, send_bytes, stream);
}

int zfpx_decode_unpack(const zfpx_plan* p, const void* d_recv, size_t recv_bytes, int rate,
                       float* d_dst, int64_t dst_elems, void* stream) {
  if (!p) return ZFPX_EINVAL;
  return do_decode_unpack(p, 0, p->nchunks, d_recv, recv_bytes, rate, d_dst, dst_elems, stream);
}

int zfpx_pack_encode_chunks(const zfpx_plan* p, int32_t first, int32_t count, const float* d_src,
                            int64_t src_elems, int rate, void* d_send, size_t send_bytes,
                            void* stream) {
  return do_pack_encode(p, first, count, d_src, src_elems, rate, d_send, send_bytes, stream);
}

int zfpx_decode_unpack_chunks(const zfpx_plan* p, int32_t first, int32_t count,
                              const void* d_recv, size_t recv_bytes, int rate, float* d_dst,
                              int64_t dst_elems, void* stream) {
  return do_decode_unpack(p, first, count, d_recv, recv_bytes, rate, d_dst, dst_elems, stream);
}

// ---------------------------------------------------------------------------
// Chunk-wise pipeline over a link
// ---------------------------------------------------------------------------

struct zfpx_pipeline {
  const zfpx_plan* plan = nullptr;
  int rate = 0;
  std::vector<int32_t> first;          // group g = chunks [first[g], first[g + 1])
  std::vector<hipEvent_t> sent, recvd;  // per group
  // end of the last send's copies / the last recv's decodes: the next call
  // of the same kind waits for them before it overwrites the buffers
  hipEvent_t send_done = nullptr, recv_done = nullptr;
};

int zfpx_pipeline_destroy(zfpx_pipeline* pp) {
  if (!pp) return ZFPX_EINVAL;
  for (hipEvent_t e : pp->sent)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : pp->recvd)
    if (e) (void)hipEventDestroy(e);
  if (pp->send_done) (void)hipEventDestroy(pp->send_done);
  if (pp->recv_done) (void)hipEventDestroy(pp->recv_done);
  delete pp;
  return ZFPX_OK;
}

int zfpx_pipeline_create(const zfpx_plan* p, int rate, int32_t groups, zfpx_pipeline** out) {
  if (!p || !out || !rate_ok(rate) || groups < 1) return ZFPX_EINVAL;
  *out = nullptr;
  const int32_t g = std::min<int32_t>(groups, std::max<int32_t>(p->nchunks, 1));
  zfpx_pipeline* pp = new (std::nothrow) zfpx_pipeline();
  if (!pp) return ZFPX_ENOMEM;
  pp->plan = p;
  pp->rate = rate;
  pp->first.resize(g + 1);
  for (int32_t i = 0; i <= g; i++) pp->first[i] = (int32_t)((int64_t)i * p->nchunks / g);
  pp->sent.assign(g, nullptr);
  pp->recvd.assign(g, nullptr);
  if (hipEventCreateWithFlags(&pp->send_done, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&pp->recv_done, hipEventDisableTiming) != hipSuccess) {
    zfpx_pipeline_destroy(pp);
    return ZFPX_EHIP;
  }
  for (int32_t i = 0; i < g; i++) {
    if (hipEventCreateWithFlags(&pp->sent[i], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&pp->recvd[i], hipEventDisableTiming) != hipSuccess) {
      zfpx_pipeline_destroy(pp);
      return ZFPX_EHIP;
    }
  }
  *out = pp;
  return ZFPX_OK;
}

// Byte range of group i's chunks in a fixed-rate stream.
static void group_bytes(const zfpx_pipeline* pp, size_t i, size_t* off, size_t* bytes) {
  const zfpx_plan* p = pp->plan;
  const int64_t b0 = p->chunk_first[pp->first[i]], b1 = p->chunk_first[pp->first[i + 1]];
  *off = (size_t)b0 * 8 * pp->rate;
  *bytes = (size_t)(b1 - b0) * 8 * pp->rate;
}

int zfpx_pipeline_send(zfpx_pipeline* pp, const float* d_src, int64_t src_elems, void* d_send,
                       size_t send_bytes, void* h_link, size_t link_bytes, void* compute_stream,
                       void* copy_stream) {
  if (!pp || !d_send || !h_link) return ZFPX_EINVAL;
  const size_t total = (size_t)pp->plan->nblocks * 8 * pp->rate;
  if (send_bytes < total || link_bytes < total) return ZFPX_ENOSPC;
  hipStream_t cs = (hipStream_t)compute_stream, xs = (hipStream_t)copy_stream;
  // d_send is rewritten below: the previous send's copies must be done
  if (hipStreamWaitEvent(cs, pp->send_done, 0) != hipSuccess) return ZFPX_EHIP;
  for (size_t i = 0; i + 1 < pp->first.size(); i++) {
    const int32_t c0 = pp->first[i], n = pp->first[i + 1] - c0;
    int st = zfpx_pack_encode_chunks(pp->plan, c0, n, d_src, src_elems, pp->rate, d_send,
                                     send_bytes, cs);
    if (st) return st;
    size_t off, bytes;
    group_bytes(pp, i, &off, &bytes);
    if (bytes == 0) continue;
    if (hipEventRecord(pp->sent[i], cs) != hipSuccess ||
        hipStreamWaitEvent(xs, pp->sent[i], 0) != hipSuccess ||
        hipMemcpyAsync((char*)h_link + off, (const char*)d_send + off, bytes,
                       hipMemcpyDeviceToHost, xs) != hipSuccess)
      return ZFPX_EHIP;
  }
  return hipEventRecord(pp->send_done, xs) == hipSuccess ? ZFPX_OK : ZFPX_EHIP;
}

int zfpx_pipeline_recv(zfpx_pipeline* pp, const void* h_link, size_t link_bytes, void* d_recv,
                       size_t recv_bytes, float* d_dst, int64_t dst_elems, void* compute_stream,
                       void* copy_stream) {
  if (!pp || !d_recv || !h_link) return ZFPX_EINVAL;
  const size_t total = (size_t)pp->plan->nblocks * 8 * pp->rate;
  if (recv_bytes < total || link_bytes < total) return ZFPX_ENOSPC;
  hipStream_t cs = (hipStream_t)compute_stream, xs = (hipStream_t)copy_stream;
  // d_recv is rewritten below: the previous recv's decodes must be done
  if (hipStreamWaitEvent(xs, pp->recv_done, 0) != hipSuccess) return ZFPX_EHIP;
  for (size_t i = 0; i + 1 < pp->first.size(); i++) {
    const int32_t c0 = pp->first[i], n = pp->first[i + 1] - c0;
    size_t off, bytes;
    group_bytes(pp, i, &off, &bytes);
    if (bytes == 0) continue;
    if (hipMemcpyAsync((char*)d_recv + off, (const char*)h_link + off, bytes,
                       hipMemcpyHostToDevice, xs) != hipSuccess ||
        hipEventRecord(pp->recvd[i], xs) != hipSuccess ||
        hipStreamWaitEvent(cs, pp->recvd[i], 0) != hipSuccess)
      return ZFPX_EHIP;
    int st = zfpx_decode_unpack_chunks(pp->plan, c0, n, d_recv, recv_bytes, pp->rate, d_dst,
                                       dst_elems, cs);
    if (st) return st;
  }
  return hipEventRecord(pp->recv_done, cs) == hipSuccess ? ZFPX_OK : ZFPX_EHIP;
}

// ---------------------------------------------------------------------------
// Variable-size modes
// ---------------------------------------------------------------------------

static bool var_params_ok(int maxprec, int minexp, int rate_cap) {
  return maxprec >= 1 && maxprec <= 32 && minexp >= ZFPX_MINEXP_NONE && minexp <= 1024 &&
         rate_ok(rate_cap);
}

int zfpx_accuracy_minexp(double tolerance) {
  if (!(tolerance > 0) || tolerance != tolerance) return ZFPX_MINEXP_NONE;
  int e = 0;
  (void)frexp(tolerance, &e);  // tolerance = f 2^e, f in [1/2, 1)
  return e - 1;
}

int zfpx_plan_var_sizes(const zfpx_plan* p, int rate_cap, int64_t* max_words, int64_t* ntiles,
                        size_t* work_bytes) {
  if (!p || !rate_ok(rate_cap)) return ZFPX_EINVAL;
  if (max_words) *max_words = p->nblocks * 2 * rate_cap;
  if (ntiles) *ntiles = (p->nblocks + 63) / 64;
  if (work_bytes)
    *work_bytes = (var_stage_words(p->nblocks, rate_cap) + (size_t)(p->nblocks + 63) / 64) *
                  sizeof(uint32_t);
  return ZFPX_OK;
}

int zfpx_plan_encode_var(const zfpx_plan* p, const float* d_src, int64_t src_elems, int maxprec,
                         int minexp, int rate_cap, uint32_t* d_words, size_t words_bytes,
                         uint8_t* d_nd, int64_t* d_tile_off, void* d_work, size_t work_bytes,
                         void* stream) {
  if (!p || !var_params_ok(maxprec, minexp, rate_cap)) return ZFPX_EINVAL;
  if (p->nblocks == 0) return ZFPX_OK;
  if (!d_src || !d_words || !d_nd || !d_tile_off || !d_work || !aligned(d_words, 4) ||
      !aligned(d_tile_off, 8) || !aligned(d_work, 4) || src_elems < p->min_elems)
    return ZFPX_EINVAL;
  const size_t stage = var_stage_words(p->nblocks, rate_cap);
  if (work_bytes < (stage + (size_t)(p->nblocks + 63) / 64) * sizeof(uint32_t))
    return ZFPX_ENOSPC;
  bool vec4 = p->vec4 && aligned(d_src, 16);
  uint32_t* w = (uint32_t*)d_work;
  hipError_t e = launch_plan_encode_var(p->dev, vec4, d_src, d_words, words_bytes / 4, d_nd,
                                        d_tile_off, w, w + stage, rate_cap, (int32_t)p->nblocks,
                                        maxprec, minexp, (hipStream_t)stream);
  return e == hipSuccess ? ZFPX_OK : ZFPX_EHIP;
}

int zfpx_plan_encode_var_noalloc(const zfpx_plan* p, const float* d_src, int64_t src_elems,
                                 int maxprec, int minexp, int rate_cap, uint32_t* d_words,
                                 size_t words_bytes, uint8_t* d_nd, int64_t* d_tile_off,
                                 void* stream) {
  if (!p || !var_params_ok(maxprec, minexp, rate_cap)) return ZFPX_EINVAL;
  if (p->nblocks == 0) return ZFPX_OK;
  const size_t need =
      (var_stage_words(p->nblocks, rate_cap) + (size_t)(p->nblocks + 63) / 64) * sizeof(uint32_t);
  if (need > kNoAllocScratchBytes) return ZFPX_ENOSPC;
  void* work = nullptr;
  if (noalloc_scratch(&work) != hipSuccess) return ZFPX_EHIP;
  return zfpx_plan_encode_var(p, d_src, src_elems, maxprec, minexp, rate_cap, d_words,
                              words_bytes, d_nd, d_tile_off, work, kNoAllocScratchBytes, stream);
}

size_t zfpx_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

int zfpx_plan_decode_var(const zfpx_plan* p, const uint32_t* d_words, size_t words_bytes,
                         const uint8_t* d_nd, const int64_t* d_tile_off, int maxprec, int minexp,
                         int rate_cap, float* d_dst, int64_t dst_elems, void* stream) {
  if (!p || !var_params_ok(maxprec, minexp, rate_cap)) return ZFPX_EINVAL;
  if (p->nblocks == 0) return ZFPX_OK;
  if (!d_words || !d_nd || !d_tile_off || !d_dst || !aligned(d_words, 4) ||
      !aligned(d_tile_off, 8) || dst_elems < p->min_elems)
    return ZFPX_EINVAL;
  bool vec4 = p->vec4 && aligned(d_dst, 16);
  hipError_t e = launch_plan_decode_var(p->dev, vec4, d_words, words_bytes / 4, d_nd, d_tile_off,
                                        d_dst, rate_cap, (int32_t)p->nblocks, maxprec, minexp,
                                        (hipStream_t)stream);
  return e == hipSuccess ? ZFPX_OK : ZFPX_EHIP;
}

int zfpx_plan_var_chunk_offsets(const zfpx_plan* p, const uint8_t* d_nd,
                                const int64_t* d_tile_off, int64_t* d_chunk_off, void* stream) {
  if (!p || !d_chunk_off || !aligned(d_chunk_off, 8)) return ZFPX_EINVAL;
  if (p->nblocks > 0 && (!d_nd || !d_tile_off || !aligned(d_tile_off, 8))) return ZFPX_EINVAL;
  if (p->nblocks == 0) {
    hipError_t e = launch_fill_u64((uint64_t*)d_chunk_off, p->nchunks + 1, 0,
                                   (hipStream_t)stream);
    return e == hipSuccess ? ZFPX_OK : ZFPX_EHIP;
  }
  hipError_t e = launch_var_chunk_offsets(p->d_chunk_first, p->nchunks, d_nd, d_tile_off,
                                          d_chunk_off, (hipStream_t)stream);
  return e == hipSuccess ? ZFPX_OK : ZFPX_EHIP;
}

// ---------------------------------------------------------------------------
// Launch configuration and autotuning
// ---------------------------------------------------------------------------

int zfpx_plan_set_config(zfpx_plan* p, int op, int rate, int wg_threads, int grid_wgs) {
  if (!p || (op != kOpEncode && op != kOpDecode) || rate < 0 || rate > 32) return ZFPX_EINVAL;
  LaunchCfg c;
  c.wg = wg_threads;
  c.grid = grid_wgs;
  if (!cfg_ok(c, rate == 0 ? 1 : rate)) return ZFPX_EINVAL;
  p->cfg[{op, rate}] = c;
  return ZFPX_OK;
}

int zfpx_plan_get_config(const zfpx_plan* p, int op, int rate, int* wg_threads, int* grid_wgs) {
  if (!p || (op != kOpEncode && op != kOpDecode) || !rate_ok(rate)) return ZFPX_EINVAL;
  LaunchCfg c = p->config(op, rate);
  if (wg_threads) *wg_threads = c.wg;
  if (grid_wgs) *grid_wgs = c.grid;
  return ZFPX_OK;
}

static std::string tune_key(const zfpx_plan* p, int op, int rate) {
  int dev = 0;
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    arch = prop.gcnArchName;
  for (char& ch : arch)
    if (ch == ' ' || ch == ':') ch = '_';
  char buf[256];
  snprintf(buf, sizeof buf, "%s op%d r%d c%lld b%lld v%lld s%lld", arch.c_str(), op, rate,
           (long long)p->shape_key[0], (long long)p->shape_key[1], (long long)p->shape_key[2],
           (long long)p->shape_key[3]);
  return buf;
}

static bool cache_lookup(const char* path, const std::string& key, LaunchCfg* c) {
  if (!path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (fgets(line, sizeof line, f)) {
    char* bar = strchr(line, '|');
    if (!bar) continue;
    std::string k(line, bar - line);
    int wg = 0, grid = 0;
    if (k == key && sscanf(bar + 1, "%d %d", &wg, &grid) == 2) {
      c->wg = wg;
      c->grid = grid;
      found = true;  // the last entry wins
    }
  }
  fclose(f);
  return found;
}

static void cache_store(const char* path, const std::string& key, LaunchCfg c, double us) {
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s|%d %d %.3f\n", key.c_str(), c.wg, c.grid, us);
  fclose(f);
}

int zfpx_autotune(zfpx_plan* p, int op, int rate, const float* d_src, int64_t src_elems,
                  void* d_stream_buf, size_t stream_bytes, float* d_dst, int64_t dst_elems,
                  const char* cache_path, void* stream, double* best_us) {
  if (!p || !rate_ok(rate) || (op != kOpEncode && op != kOpDecode)) return ZFPX_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  std::string key = tune_key(p, op, rate);
  LaunchCfg cached;
  if (cache_lookup(cache_path, key, &cached) && cfg_ok(cached, rate)) {
    p->cfg[{op, rate}] = cached;
    if (best_us) *best_us = -1.0;
    return ZFPX_OK;
  }
  int cus = device_cu_count();
  std::vector<LaunchCfg> cands;
  for (int wg : {64, 128, 256})
    for (int mult : {0, 1, 2, 4, 8, 16}) {
      LaunchCfg c;
      c.wg = wg;
      c.grid = mult == 0 ? 0 : mult * cus * 4 / (wg / 64);  // waves per CU = 4 * mult
      if (cfg_ok(c, rate)) cands.push_back(c);
    }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return ZFPX_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return ZFPX_EHIP;
  }
  auto saved = p->cfg;
  double best = 1e300;
  LaunchCfg best_c = default_cfg(op, p->nblocks);
  int st = ZFPX_OK;
  for (const LaunchCfg& c : cands) {
    p->cfg[{op, rate}] = c;
    auto run = [&]() {
      return op == kOpEncode
                 ? zfpx_pack_encode(p, d_src, src_elems, rate, d_stream_buf, stream_bytes, s)
                 : zfpx_decode_unpack(p, d_stream_buf, stream_bytes, rate, d_dst, dst_elems, s);
    };
    for (int i = 0; i < 2 && st == ZFPX_OK; i++) st = run();
    if (st) break;
    const int reps = 5;
    if (hipEventRecord(e0, s) != hipSuccess) { st = ZFPX_EHIP; break; }
    for (int i = 0; i < reps && st == ZFPX_OK; i++) st = run();
    if (st) break;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      st = ZFPX_EHIP;
      break;
    }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    double us = 1000.0 * ms / reps;
    if (us < best) {
      best = us;
      best_c = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) {
    p->cfg = saved;
    return st;
  }
  p->cfg[{op, rate}] = best_c;
  cache_store(cache_path, key, best_c, best);
  if (best_us) *best_us = best;
  return ZFPX_OK;
}

// ---------------------------------------------------------------------------
// Graphs
// ---------------------------------------------------------------------------

int zfpx_graph_destroy(zfpx_graph* g) {
  if (!g) return ZFPX_EINVAL;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return ZFPX_OK;
}

int zfpx_graph_create(const zfpx_plan* p, int rate, const float* d_src, int64_t src_elems,
                      void* d_send, size_t send_bytes, float* d_dst, int64_t dst_elems,
                      zfpx_graph** out) {
  if (!p || !out || !rate_ok(rate)) return ZFPX_EINVAL;
  *out = nullptr;
  if (!d_src || !d_send || !d_dst) return ZFPX_EINVAL;
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return ZFPX_EHIP;
  zfpx_graph* g = new (std::nothrow) zfpx_graph();
  if (!g) {
    (void)hipStreamDestroy(cs);
    return ZFPX_ENOMEM;
  }
  int st = ZFPX_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    st = ZFPX_EHIP;
  } else {
    st = zfpx_pack_encode(p, d_src, src_elems, rate, d_send, send_bytes, cs);
    if (st == ZFPX_OK)
      st = zfpx_decode_unpack(p, d_send, send_bytes, rate, d_dst, dst_elems, cs);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &graph);
    g->graph = graph;
    if (st == ZFPX_OK && e != hipSuccess) st = ZFPX_EHIP;
    if (st == ZFPX_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
      st = ZFPX_EHIP;
  }
  (void)hipStreamDestroy(cs);
  if (st) {
    zfpx_graph_destroy(g);
    return st;
  }
  *out = g;
  return ZFPX_OK;
}

int zfpx_graph_launch(zfpx_graph* g, void* stream) {
  if (!g || !g->exec) return ZFPX_EINVAL;
  return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? ZFPX_OK : ZFPX_EHIP;
}

// ---------------------------------------------------------------------------
// float16 comparator
// ---------------------------------------------------------------------------

int f16_truncate(const float* d_in, size_t n, uint16_t* d_out, void* stream) {
  if (n == 0) return ZFPX_OK;
  if (!d_in || !d_out || !aligned(d_in, 4) || !aligned(d_out, 2)) return ZFPX_EINVAL;
  return launch_f16_truncate(d_in, n, d_out, (hipStream_t)stream) == hipSuccess ? ZFPX_OK
                                                                                 : ZFPX_EHIP;
}

int f16_restore(const uint16_t* d_in, size_t n, float* d_out, void* stream) {
  if (n == 0) return ZFPX_OK;
  if (!d_in || !d_out || !aligned(d_in, 2) || !aligned(d_out, 4)) return ZFPX_EINVAL;
  return launch_f16_restore(d_in, n, d_out, (hipStream_t)stream) == hipSuccess ? ZFPX_OK
                                                                                : ZFPX_EHIP;
}

}  // extern "C"
