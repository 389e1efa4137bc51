// server.cpp -- continuous-batching serving runtime around the device loop.
//
// Requests (compress or decompress a regular float32 array at some rate) are
// queued on the host and admitted in arrival order while a ring slot is free
// and the bytes they touch (input + output) fit in the HBM budget.  Admission
// writes the request's descriptor into the ring (host-coherent memory) and
// publishes it; the device loop (k_serve) picks it up at once, splits it into
// 64-block tiles and interleaves them with the tiles of every other request
// in flight.  Completion flags come back through host memory; the host
// timestamps them, frees the budget and admits more.  The device loop is
// (re)launched whenever requests are in flight and no loop is running.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/zfpx.h"
#include "internal.hpp"

using namespace zfpx;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

int64_t ceil4(int64_t n) { return (n + 3) / 4; }

struct Pending {
  uint64_t ticket;
  zfpx_request rq;
  int64_t nblocks;
  size_t bytes;
  double t_submit;
};

struct SlotState {
  bool active = false;
  uint64_t seq = 0;
  uint64_t ticket = 0;
  size_t bytes = 0;
  int64_t ntiles = 0;
  double t_submit = 0;
};

struct Result {
  bool done = false;
  double latency = 0;
};

bool request_ok(const zfpx_request* rq, int64_t* nblocks, size_t* bytes) {
  if (!rq || (rq->op != 0 && rq->op != 1) || rq->rate < 1 || rq->rate > 32) return false;
  if (rq->nx < 1 || rq->ny < 1 || rq->nz < 1 || !rq->d_in || !rq->d_out) return false;
  int64_t nb = ceil4(rq->nx) * ceil4(rq->ny) * ceil4(rq->nz);
  if (nb > 0x7fffffffLL) return false;
  const void* words = rq->op == 0 ? rq->d_out : rq->d_in;
  if (((uintptr_t)words & 7) != 0) return false;
  *nblocks = nb;
  *bytes = (size_t)(rq->nx * rq->ny * rq->nz * 4) + (size_t)nb * 8 * rq->rate;
  return true;
}

// Byte span of the request's float32 array when the device loop may move it
// in 16-byte pieces through a 32-bit offset (unit x stride, rows 16-byte
// aligned, non-negative strides, span below 4 GiB); 0 otherwise.
uint32_t vector_span(const zfpx_request* rq) {
  const void* f = rq->op == 0 ? rq->d_in : rq->d_out;
  if (rq->sx != 1 || (rq->sy & 3) != 0 || (rq->sz & 3) != 0 || ((uintptr_t)f & 15) != 0)
    return 0;
  if (rq->sy < 0 || rq->sz < 0) return 0;
  const int64_t last = (rq->nx - 1) + (rq->ny - 1) * rq->sy + (rq->nz - 1) * rq->sz;
  const int64_t bytes = 4 * (last + 1);
  if (bytes <= 0 || bytes > 0xffffffffLL) return 0;
  return (uint32_t)bytes;
}

}  // namespace

struct zfpx_server {
  std::mutex mu;
  size_t budget = 0, inflight = 0, max_inflight = 0;
  int cap = 0;
  size_t max_queue = 0;
  int workgroups = 0;
  ServeCtl* ctl = nullptr;  // host-coherent
  ServeDesc* ring = nullptr;
  uint64_t* flags = nullptr;
  ServeCtl* ctl_d = nullptr;
  ServeDesc* ring_d = nullptr;
  uint64_t* flags_d = nullptr;
  uint64_t* claim = nullptr;  // device memory
  uint64_t* done = nullptr;
  ServeDevCtl* dctl = nullptr;
  ServeDesc* ring_dev = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t loop_done = nullptr;
  bool loop_running = false;
  uint64_t launches = 0;
  uint64_t next_seq = 0, next_ticket = 1;
  std::deque<Pending> queue;
  std::vector<SlotState> slots;
  std::unordered_map<uint64_t, Result> results;
  // requests low_seq .. next_seq-1 may be in flight (at most cap of them)
  uint64_t low_seq = 0;
  size_t nactive = 0;
  int64_t inflight_tiles = 0;  // tiles of the requests in flight
  double last_query = 0;  // last time the device loop's end was queried
  // tickets completed since the last look, gathered while collect_done is set
  bool collect_done = false;
  std::vector<uint64_t> completed;
  uint64_t idle_ticks = 0, max_ticks = 0;
  uint64_t ticks_per_ms = 0;  // device wall clock
  int device = 0;
};

static void server_free(zfpx_server* sv) {
  if (sv->stream) {
    if (sv->ctl) __atomic_store_n(&sv->ctl->stop, 1u, __ATOMIC_SEQ_CST);
    (void)hipStreamSynchronize(sv->stream);
  }
  if (sv->loop_done) (void)hipEventDestroy(sv->loop_done);
  if (sv->stream) (void)hipStreamDestroy(sv->stream);
  if (sv->claim) (void)hipFree(sv->claim);
  if (sv->done) (void)hipFree(sv->done);
  if (sv->dctl) (void)hipFree(sv->dctl);
  if (sv->ring_dev) (void)hipFree(sv->ring_dev);
  if (sv->ctl) (void)hipHostFree(sv->ctl);
  if (sv->ring) (void)hipHostFree(sv->ring);
  if (sv->flags) (void)hipHostFree(sv->flags);
  delete sv;
}

// Launch the device loop if requests are in flight and none is running.
static int ensure_loop(zfpx_server* sv) {
  if (sv->nactive == 0) return ZFPX_OK;
  if (sv->loop_running) {
    // the loop leaves only after an idle spell: asking the runtime at every
    // host pass would cost more than it tells
    const double t = now_s();
    if (t - sv->last_query < 20e-6) return ZFPX_OK;
    sv->last_query = t;
    hipError_t q = hipEventQuery(sv->loop_done);
    if (q == hipErrorNotReady) return ZFPX_OK;
    if (q != hipSuccess) return ZFPX_EHIP;
    sv->loop_running = false;
  }
  ServeDev d;
  d.ctl = sv->ctl_d;
  d.ring = sv->ring_d;
  d.done_flag = sv->flags_d;
  d.dctl = sv->dctl;
  d.ring_dev = sv->ring_dev;
  d.claim = sv->claim;
  d.done = sv->done;
  d.cap = sv->cap;
  d.pad = 0;
  d.idle_ticks = sv->idle_ticks;
  d.max_ticks = sv->max_ticks;
  if (launch_serve(d, sv->workgroups, sv->stream) != hipSuccess) return ZFPX_EHIP;
  if (hipEventRecord(sv->loop_done, sv->stream) != hipSuccess) return ZFPX_EHIP;
  sv->loop_running = true;
  sv->launches++;
  return ZFPX_OK;
}

// Collect completions, admit queued requests, keep the loop running.
static int progress_locked(zfpx_server* sv) {
  const double t = now_s();
  for (uint64_t sq = sv->low_seq; sq < sv->next_seq; sq++) {
    const int j = (int)(sq % (uint64_t)sv->cap);
    SlotState& s = sv->slots[j];
    if (!s.active || s.seq != sq) continue;
    uint64_t f = __atomic_load_n(&sv->flags[j], __ATOMIC_ACQUIRE);
    if (f == s.seq + 1) {
      s.active = false;
      sv->nactive--;
      sv->inflight -= s.bytes;
      sv->inflight_tiles -= s.ntiles;
      Result& r = sv->results[s.ticket];
      r.done = true;
      r.latency = t - s.t_submit;
      if (sv->collect_done) sv->completed.push_back(s.ticket);
    }
  }
  while (sv->low_seq < sv->next_seq) {
    const SlotState& s = sv->slots[sv->low_seq % (uint64_t)sv->cap];
    if (s.active && s.seq == sv->low_seq) break;
    sv->low_seq++;
  }
  uint64_t oldest = sv->low_seq;
  while (!sv->queue.empty()) {
    Pending& p = sv->queue.front();
    int j = (int)(sv->next_seq % (uint64_t)sv->cap);
    if (sv->slots[j].active || sv->inflight + p.bytes > sv->budget) break;
    ServeDesc q{};
    q.seq = sv->next_seq;
    q.op = p.rq.op;
    q.rate = p.rq.rate;
    q.nblocks = (int32_t)p.nblocks;
    q.ntiles = (int32_t)((p.nblocks + 63) / 64);
    q.vspan = vector_span(&p.rq);
    // Tiles are handed out in runs of up to 8 per wavefront per claim (a
    // worker workgroup claims one run for each of its wavefronts), by load:
    // with k requests in flight a request's fair share of the W worker
    // wavefronts is about W / k, and runs of ntiles * k / (2 W) tiles give it
    // that many claims' worth of spread; but a share by tiles is what counts
    // when the others are small, so the run is also at most T / (2 W), T the
    // tiles in flight with this request's.  A lone request is spread one
    // tile per wavefront over every workgroup (lowest latency); under load,
    // longer runs cut claim and descriptor traffic.
    {
      const int64_t workers = std::max<int64_t>(1, (int64_t)(sv->workgroups - 1) * kServeWaves);
      const int64_t by_count = (int64_t)q.ntiles * (int64_t)(sv->nactive + 1) / (2 * workers);
      const int64_t by_tiles = (sv->inflight_tiles + q.ntiles) / (2 * workers);
      const int64_t run = std::min(by_count, by_tiles);
      q.per_claim = (int32_t)std::min<int64_t>(8, std::max<int64_t>(1, run));
    }
    q.geo = RegularDev{p.rq.nx, p.rq.ny, p.rq.nz, p.rq.sx, p.rq.sy, p.rq.sz,
                       (int32_t)ceil4(p.rq.nx), (int32_t)ceil4(p.rq.ny)};
    q.in = (uint64_t)(uintptr_t)p.rq.d_in;
    q.out = (uint64_t)(uintptr_t)p.rq.d_out;
    memcpy(&sv->ring[j], &q, sizeof q);
    SlotState& s = sv->slots[j];
    s.active = true;
    sv->nactive++;
    s.seq = q.seq;
    s.ticket = p.ticket;
    s.bytes = p.bytes;
    s.ntiles = q.ntiles;
    s.t_submit = p.t_submit;
    sv->inflight += p.bytes;
    sv->inflight_tiles += q.ntiles;
    if (sv->inflight > sv->max_inflight) sv->max_inflight = sv->inflight;
    if (q.seq < oldest) oldest = q.seq;
    sv->next_seq++;
    std::atomic_thread_fence(std::memory_order_release);
    __atomic_store_n(&sv->ctl->published, sv->next_seq, __ATOMIC_RELEASE);
    sv->queue.pop_front();
  }
  __atomic_store_n(&sv->ctl->oldest, oldest, __ATOMIC_RELEASE);
  return ensure_loop(sv);
}

extern "C" {

int zfpx_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t workgroups,
                       zfpx_server** out) {
  if (!out || hbm_budget_bytes == 0 || max_slots < 1 || max_slots > 65536 || workgroups < 0)
    return ZFPX_EINVAL;
  *out = nullptr;
  zfpx_server* sv = new (std::nothrow) zfpx_server();
  if (!sv) return ZFPX_ENOMEM;
  sv->budget = hbm_budget_bytes;
  sv->cap = max_slots;
  sv->max_queue = (size_t)1 << 20;
  sv->slots.resize(max_slots);
  if (hipGetDevice(&sv->device) != hipSuccess) {
    delete sv;
    return ZFPX_EHIP;
  }
  // one workgroup of eight wavefronts per compute unit (two wavefronts per
  // SIMD, as many as the LDS slices of rate-32 tiles allow); workgroup 0 only
  // dispatches, so at least one more is needed
  sv->workgroups = workgroups > 0 ? std::max(2, workgroups) : device_cu_count();
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, sv->device) != hipSuccess ||
      khz <= 0)
    khz = 100000;  // 100 MHz
  sv->ticks_per_ms = (uint64_t)khz;
  sv->idle_ticks = (uint64_t)khz * 2;         // 2 ms in which nothing is published
  sv->max_ticks = (uint64_t)khz * 1000 * 60;  // 60 s per launch at most
  unsigned fl = hipHostMallocCoherent | hipHostMallocMapped;
  if (hipHostMalloc((void**)&sv->ctl, sizeof(ServeCtl), fl) != hipSuccess ||
      hipHostMalloc((void**)&sv->ring, sizeof(ServeDesc) * max_slots, fl) != hipSuccess ||
      hipHostMalloc((void**)&sv->flags, sizeof(uint64_t) * max_slots, fl) != hipSuccess) {
    server_free(sv);
    return ZFPX_ENOMEM;
  }
  memset(sv->ctl, 0, sizeof(ServeCtl));
  memset(sv->ring, 0xff, sizeof(ServeDesc) * max_slots);  // seq = ~0: no request yet
  memset(sv->flags, 0, sizeof(uint64_t) * max_slots);
  if (hipHostGetDevicePointer((void**)&sv->ctl_d, sv->ctl, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&sv->ring_d, sv->ring, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&sv->flags_d, sv->flags, 0) != hipSuccess) {
    server_free(sv);
    return ZFPX_EHIP;
  }
  if (hipMalloc((void**)&sv->claim, sizeof(uint64_t) * max_slots) != hipSuccess ||
      hipMalloc((void**)&sv->done, sizeof(uint64_t) * max_slots) != hipSuccess ||
      hipMalloc((void**)&sv->dctl, sizeof(ServeDevCtl)) != hipSuccess ||
      hipMalloc((void**)&sv->ring_dev, sizeof(ServeDesc) * max_slots) != hipSuccess) {
    server_free(sv);
    return ZFPX_ENOMEM;
  }
  {
    ServeDevCtl z{0, 0, 0};
    std::vector<ServeDesc> blank(max_slots);
    memset(blank.data(), 0xff, sizeof(ServeDesc) * max_slots);
    if (hipMemcpy(sv->dctl, &z, sizeof z, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(sv->ring_dev, blank.data(), sizeof(ServeDesc) * max_slots,
                  hipMemcpyHostToDevice) != hipSuccess) {
      server_free(sv);
      return ZFPX_EHIP;
    }
  }
  // claim and done counters: (request number << 32) | count, all starting
  // at request 0 with count 0 (later requests move them on with an atomic max)
  std::vector<uint64_t> init(max_slots, 0);
  if (hipMemcpy(sv->claim, init.data(), sizeof(uint64_t) * max_slots, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(sv->done, init.data(), sizeof(uint64_t) * max_slots, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&sv->loop_done, hipEventDisableTiming) != hipSuccess) {
    server_free(sv);
    return ZFPX_EHIP;
  }
  *out = sv;
  return ZFPX_OK;
}

int zfpx_server_submit(zfpx_server* sv, const zfpx_request* rq, uint64_t* ticket) {
  if (!sv || !ticket) return ZFPX_EINVAL;
  int64_t nb;
  size_t bytes;
  if (!request_ok(rq, &nb, &bytes) || bytes > sv->budget) return ZFPX_EINVAL;
  std::lock_guard<std::mutex> g(sv->mu);
  // request numbers tag the device counters in 32 bits and must not wrap
  if (sv->next_seq + sv->queue.size() >= 0xffffffffULL) return ZFPX_ESTATE;
  if (sv->queue.size() >= sv->max_queue) return ZFPX_EAGAIN;
  Pending p{sv->next_ticket++, *rq, nb, bytes, now_s()};
  *ticket = p.ticket;
  sv->results[p.ticket] = Result{};
  sv->queue.push_back(p);
  return progress_locked(sv);
}

int zfpx_server_progress(zfpx_server* sv) {
  if (!sv) return ZFPX_EINVAL;
  std::lock_guard<std::mutex> g(sv->mu);
  return progress_locked(sv);
}

int zfpx_server_poll(zfpx_server* sv, uint64_t ticket, int* done, double* latency_s) {
  if (!sv || !done) return ZFPX_EINVAL;
  std::lock_guard<std::mutex> g(sv->mu);
  int st = progress_locked(sv);
  if (st) return st;
  auto it = sv->results.find(ticket);
  if (it == sv->results.end()) return ZFPX_EINVAL;
  *done = it->second.done ? 1 : 0;
  if (latency_s) *latency_s = it->second.latency;
  if (it->second.done) sv->results.erase(it);
  return ZFPX_OK;
}

int zfpx_server_drain(zfpx_server* sv, double timeout_s) {
  if (!sv) return ZFPX_EINVAL;
  const double t_end = now_s() + timeout_s;
  for (;;) {
    {
      std::lock_guard<std::mutex> g(sv->mu);
      int st = progress_locked(sv);
      if (st) return st;
      if (sv->queue.empty() && sv->nactive == 0) return ZFPX_OK;
    }
    if (now_s() > t_end) return ZFPX_EAGAIN;
    std::this_thread::yield();
  }
}

int zfpx_server_stats(zfpx_server* sv, uint64_t* completed, size_t* max_inflight_bytes,
                      uint64_t* loop_launches) {
  if (!sv) return ZFPX_EINVAL;
  std::lock_guard<std::mutex> g(sv->mu);
  if (completed) *completed = sv->next_seq;
  if (max_inflight_bytes) *max_inflight_bytes = sv->max_inflight;
  if (loop_launches) *loop_launches = sv->launches;
  return ZFPX_OK;
}

int zfpx_server_set_max_queue(zfpx_server* sv, size_t max_queued) {
  if (!sv || max_queued < 1 || max_queued > ((size_t)1 << 20)) return ZFPX_EINVAL;
  std::lock_guard<std::mutex> g(sv->mu);
  sv->max_queue = max_queued;
  return ZFPX_OK;
}

int zfpx_server_set_idle_us(zfpx_server* sv, uint64_t idle_us) {
  if (!sv || idle_us < 100 || idle_us > 10000000) return ZFPX_EINVAL;
  std::lock_guard<std::mutex> g(sv->mu);
  // taken by the next launch of the loop
  sv->idle_ticks = idle_us * sv->ticks_per_ms / 1000;
  return ZFPX_OK;
}

int zfpx_server_destroy(zfpx_server* sv) {
  if (!sv) return ZFPX_EINVAL;
  server_free(sv);
  return ZFPX_OK;
}

int zfpx_server_replay(zfpx_server* sv, const zfpx_request* rq, const double* arrival_s,
                       int64_t n, double timeout_s, double* latency_s) {
  if (!sv || (n > 0 && (!rq || !arrival_s || !latency_s))) return ZFPX_EINVAL;
  std::vector<uint64_t> tickets(n, 0);
  std::unordered_map<uint64_t, int64_t> index;
  const double t0 = now_s();
  int64_t next = 0, finished = 0;
  while (finished < n) {
    const double t = now_s() - t0;
    if (t > timeout_s) return ZFPX_EAGAIN;
    {
      std::lock_guard<std::mutex> g(sv->mu);
      while (next < n && arrival_s[next] <= t) {
        int64_t nb;
        size_t bytes;
        if (!request_ok(&rq[next], &nb, &bytes) || bytes > sv->budget) return ZFPX_EINVAL;
        Pending p{sv->next_ticket++, rq[next], nb, bytes, t0 + arrival_s[next]};
        sv->results[p.ticket] = Result{};
        index[p.ticket] = next;
        sv->queue.push_back(p);
        next++;
      }
      sv->collect_done = true;
      int st = progress_locked(sv);
      sv->collect_done = false;
      if (st) {
        sv->completed.clear();
        return st;
      }
      for (uint64_t tk : sv->completed) {
        auto it = index.find(tk);
        if (it == index.end()) continue;  // a request submitted outside the replay
        auto r = sv->results.find(tk);
        latency_s[it->second] = r->second.latency;
        sv->results.erase(r);
        index.erase(it);
        finished++;
      }
      sv->completed.clear();
    }
  }
  return ZFPX_OK;
}

int zfpx_plain_replay(const zfpx_request* rq, const double* arrival_s, int64_t n,
                      double timeout_s, void* stream, double* latency_s) {
  if (n > 0 && (!rq || !arrival_s || !latency_s)) return ZFPX_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int pool = 1024;
  std::vector<hipEvent_t> ev(pool, nullptr);
  for (int i = 0; i < pool; i++)
    if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess) {
      for (int k = 0; k < i; k++) (void)hipEventDestroy(ev[k]);
      return ZFPX_EHIP;
    }
  const double t0 = now_s();
  int64_t next = 0, finished = 0;
  int st = ZFPX_OK;
  while (finished < n && st == ZFPX_OK) {
    const double t = now_s() - t0;
    if (t > timeout_s) {
      st = ZFPX_EAGAIN;
      break;
    }
    // launch every request that has arrived (FIFO on one stream), while the
    // event pool has room
    while (next < n && arrival_s[next] <= t && next - finished < pool) {
      const zfpx_request& q = rq[next];
      int64_t nb;
      size_t bytes;
      if (!request_ok(&q, &nb, &bytes)) {
        st = ZFPX_EINVAL;
        break;
      }
      st = q.op == 0 ? zfpx_encode_fixed_rate((const float*)q.d_in, q.nx, q.ny, q.nz, q.sx, q.sy,
                                              q.sz, q.rate, q.d_out, (size_t)nb * 8 * q.rate, s)
                     : zfpx_decode_fixed_rate(q.d_in, (size_t)nb * 8 * q.rate, q.nx, q.ny, q.nz,
                                              q.sx, q.sy, q.sz, q.rate, (float*)q.d_out, s);
      if (st) break;
      if (hipEventRecord(ev[next % pool], s) != hipSuccess) {
        st = ZFPX_EHIP;
        break;
      }
      next++;
    }
    while (finished < next) {
      hipError_t e = hipEventQuery(ev[finished % pool]);
      if (e == hipErrorNotReady) break;
      if (e != hipSuccess) {
        st = ZFPX_EHIP;
        break;
      }
      latency_s[finished] = (now_s() - t0) - arrival_s[finished];
      finished++;
    }
  }
  (void)hipStreamSynchronize(s);
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  return st;
}

}  // extern "C"
