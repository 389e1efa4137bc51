/*
 * zfpx.h -- ZFP coding of spectral-transform transpose buffers on AMD
 * Instinct MI355X (gfx950): fixed rate (the paper's mode), the variable-size
 * precision and accuracy modes, the float16 comparator, batching, a serving
 * loop and a chunk-wise pipeline over a link.
 *
 * The paper this implements (Breschi & Vella, "Toward GPU-Resident Climate
 * Models: a feasibility study on lossy compression for the spherical harmonic
 * transform's communication bottleneck") compresses, on the GPU, each
 * outgoing buffer of the spectral transform's pencil transpositions just
 * before the all-to-all and decompresses it on the receiver before any
 * computation, with no host-device copies (Section I).  It uses ZFP in
 * fixed-rate mode: 4x4x4 blocks coded independently into exactly r bits per
 * value, so every message has a size known in advance (Sections II-C and
 * IV-B), and compares with casting the buffer to float16 and back (Sections I
 * and IV-F).
 *
 * Conventions common to every entry point
 *  - Device buffers are caller-owned device memory (hipMalloc or a PyTorch
 *    tensor); the library never frees them.  Host arrays are read during the
 *    call only.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Hot-path calls
 *    only validate their arguments on the host and enqueue kernels: they
 *    allocate nothing, copy nothing between host and device and never
 *    synchronise, so they may be captured into a HIP graph.
 *  - Return value: ZFPX_OK (0) or a negative zfpx_status.  On an argument
 *    error nothing is enqueued.  A fault inside an enqueued kernel surfaces
 *    at the caller's next synchronisation, as with any HIP kernel.
 *  - Rates are integers 1..32 (bits per value); a block takes 64*rate bits =
 *    `rate` 64-bit words.
 *  - Arrays are float32 with x the fastest axis.  A 3-D array of nx*ny*nz
 *    values has ceil(nx/4)*ceil(ny/4)*ceil(nz/4) blocks, numbered with the x
 *    block fastest, then y, then z; partial blocks are completed by repeating
 *    the last value along each axis (clamp to edge), and decoding writes only
 *    positions inside the array.
 *  - Non-finite inputs (inf, NaN) are outside the contract: the output is
 *    deterministic but unspecified.
 */
#ifndef ZFPX_H
#define ZFPX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum zfpx_status {
  ZFPX_OK = 0,
  ZFPX_EINVAL = -1, /* bad argument: rate, size, null or misaligned pointer */
  ZFPX_ENOSPC = -2, /* output buffer smaller than the coded size */
  ZFPX_EHIP = -3,   /* a HIP runtime call failed */
  ZFPX_ENOMEM = -4, /* a library allocation failed (plans, graphs, servers) */
  ZFPX_EAGAIN = -5, /* the serving queue is full; try again */
  ZFPX_ESTATE = -6  /* object used in the wrong state */
};

/* Human-readable name of a status code (static string). */
const char* zfpx_status_string(int status);

/* Library version as 10000*major + 100*minor + patch. */
int zfpx_version(void);

/* Number of compute units of the current device (0 if unknown). */
int zfpx_device_cus(void);

/* -------------------------------------------------------------------------
 * Regular 3-D arrays
 * ---------------------------------------------------------------------- */

/*
 * Coded size in bytes of an nx*ny*nz array at `rate` bits per value:
 * ceil(nx/4)*ceil(ny/4)*ceil(nz/4) * 8 * rate (fixed-rate mode gives every
 * block exactly 64*rate bits; paper Section II-C and Table 1).  Returns a
 * negative zfpx_status for a bad rate or negative sizes.
 */
int64_t zfpx_fixed_rate_bytes(int64_t nx, int64_t ny, int64_t nz, int rate);

/*
 * Encode a strided float32 array (element (x,y,z) at d_in[x*sx + y*sy + z*sz])
 * into `rate` words per block at d_out, blocks in order (paper Section II-C:
 * independent 4^3 blocks, lifting transform, precision reduction, exactly
 * `rate` bits per value).
 *   d_out     : device, 8-byte aligned, at least zfpx_fixed_rate_bytes(...)
 *               bytes (out_bytes); ZFPX_ENOSPC if smaller.
 *   nx,ny,nz  : >= 0; an empty array enqueues nothing.
 * The caller guarantees that every element offset is inside d_in.
 */
int zfpx_encode_fixed_rate(const float* d_in, int64_t nx, int64_t ny, int64_t nz, int64_t sx,
                           int64_t sy, int64_t sz, int rate, void* d_out, size_t out_bytes,
                           void* stream);

/*
 * Decode a stream made by zfpx_encode_fixed_rate (same dims and rate) into
 * d_out[x*sx + y*sy + z*sz]; only positions inside the array are written.
 *   d_in      : device, 8-byte aligned, in_bytes >= the coded size (ENOSPC).
 * Any bit pattern decodes without a fault (every block reads only its own
 * `rate` words).
 */
int zfpx_decode_fixed_rate(const void* d_in, size_t in_bytes, int64_t nx, int64_t ny,
                           int64_t nz, int64_t sx, int64_t sy, int64_t sz, int rate,
                           float* d_out, void* stream);

/* -------------------------------------------------------------------------
 * Transpose-buffer plans: per-destination chunks with ragged rows
 * ---------------------------------------------------------------------- */

/*
 * A plan describes how one GPU's transpose buffer is cut into per-destination
 * chunks (paper Section II-B: every rank sends a sub-array to every other rank
 * of its row or column; Table 1: each message is coded as its own array).
 *
 * Chunk c (0 <= c < nchunks) is a 3-D view of a float32 buffer:
 *   levels z = 0..levels[c]-1 at element offset chunk_base[c] + z*level_stride[c];
 *   rows r = row_start[c]..row_start[c+1]-1 at further offset row_offset[r],
 *   each of row_len[r] >= 1 contiguous points.
 * Rows are taken in groups of four in order; a group is as wide as its
 * longest row; shorter rows and missing rows/levels are padded by clamping to
 * the last point/row/level.  Chunk c has ceil(levels/4) * sum over groups of
 * ceil(width/4) blocks, numbered (level block, group, x block) with the x block
 * fastest, and its stream starts at byte 8*rate*(blocks of chunks < c): the
 * send buffer is the concatenation of the chunk streams, ready for an
 * all-to-all(v) whose counts follow from geometry alone.
 *
 * All arrays are host arrays; row_start has nchunks+1 entries starting at 0.
 * zfpx_plan_create copies them into device tables (it allocates device
 * memory and synchronises; call it outside hot loops).  Plans are immutable
 * and may be used concurrently on several streams.  Errors: EINVAL for
 * inconsistent tables or more than 2^31-1 blocks, ENOMEM/EHIP on allocation.
 */
typedef struct zfpx_plan zfpx_plan;

int zfpx_plan_create(int32_t nchunks, const int64_t* chunk_base, const int64_t* level_stride,
                     const int32_t* levels, const int32_t* row_start, const int64_t* row_offset,
                     const int32_t* row_len, zfpx_plan** out);
int zfpx_plan_destroy(zfpx_plan* plan);

/*
 * Plan facts: total blocks, real (unpadded) values, and the smallest buffer
 * size in elements that holds every chunk point (any pointer may be NULL).
 */
int zfpx_plan_info(const zfpx_plan* plan, int64_t* nblocks, int64_t* nvalues,
                   int64_t* min_buffer_elems);

/*
 * Coded sizes at `rate`: per chunk bytes and byte offsets (host arrays of
 * nchunks entries, or NULL) and the total.
 */
int zfpx_plan_sizes(const zfpx_plan* plan, int rate, int64_t* chunk_bytes,
                    int64_t* chunk_offsets, int64_t* total_bytes);

/*
 * Fused pack + encode of every chunk of `plan` read from d_src (src_elems
 * float32 elements; EINVAL if a chunk point lies beyond) into d_send
 * (8-byte aligned; ENOSPC if send_bytes is below the plan's total).  One
 * launch covers all chunks (paper Section I: compress the outgoing buffer
 * on the GPU immediately before the all-to-all).
 */
int zfpx_pack_encode(const zfpx_plan* plan, const float* d_src, int64_t src_elems, int rate,
                     void* d_send, size_t send_bytes, void* stream);

/*
 * Fused decode + unpack: the mirror of zfpx_pack_encode; writes only the
 * chunk points of d_dst (dst_elems elements).  (Paper Section I: decompress on
 * the receiving side before any local computation.)
 */
int zfpx_decode_unpack(const zfpx_plan* plan, const void* d_recv, size_t recv_bytes, int rate,
                       float* d_dst, int64_t dst_elems, void* stream);

/*
 * The same two operations restricted to chunks [first, first+count); the
 * streams are read/written at their offsets inside the whole send buffer, so
 * d_send/d_recv still point at the start of the buffer.  This is the
 * one-launch-per-chunk form, and the unit for overlapping coding with
 * sending chunk by chunk (paper Section IV-D: the serial model could be
 * pipelined).
 */
int zfpx_pack_encode_chunks(const zfpx_plan* plan, int32_t first, int32_t count,
                            const float* d_src, int64_t src_elems, int rate, void* d_send,
                            size_t send_bytes, void* stream);
int zfpx_decode_unpack_chunks(const zfpx_plan* plan, int32_t first, int32_t count,
                              const void* d_recv, size_t recv_bytes, int rate, float* d_dst,
                              int64_t dst_elems, void* stream);

/* -------------------------------------------------------------------------
 * Chunk-wise pipeline over a link
 * ---------------------------------------------------------------------- */

/*
 * The paper adds codec time before and after the exchange (t_compress +
 * t_comm + t_decompress) and notes that compressing and sending could be
 * pipelined (Section IV-D).  A pipeline cuts the plan's chunks into `groups`
 * consecutive groups (fewer if there are fewer chunks):
 *   send: group g is encoded on compute_stream, then copied device -> host
 *         (h_link, at the group's offset in the fixed-rate stream) on
 *         copy_stream, so the copy of group g overlaps the encoding of g+1;
 *   recv: group g is copied host -> device on copy_stream, then decoded on
 *         compute_stream while group g+1 is being copied.
 * The host buffer stands in for the link on a single GPU (host memory over
 * PCIe); h_link must be pinned (hipHostMalloc) for the copies to be
 * asynchronous.  Both streams must be distinct; calls only enqueue (no
 * synchronisation): the send's bytes are in h_link once copy_stream reaches
 * the call's end, the recv's floats once compute_stream does.
 * A send waits (on the device) for the previous send's copies before it
 * rewrites d_send, and a recv for the previous recv's decodes before it
 * rewrites d_recv, so calls may follow each other without host
 * synchronisation.  zfpx_pipeline_create creates 2*groups + 2 HIP events
 * (call it outside hot loops); a pipeline refers to its plan, which must
 * outlive it.
 * Errors: EINVAL (null pointers, bad rate or groups < 1), ENOSPC (a buffer
 * smaller than the coded size), the errors of the range calls.
 */
typedef struct zfpx_pipeline zfpx_pipeline;

int zfpx_pipeline_create(const zfpx_plan* plan, int rate, int32_t groups, zfpx_pipeline** out);
int zfpx_pipeline_send(zfpx_pipeline* pipe, const float* d_src, int64_t src_elems, void* d_send,
                       size_t send_bytes, void* h_link, size_t link_bytes, void* compute_stream,
                       void* copy_stream);
int zfpx_pipeline_recv(zfpx_pipeline* pipe, const void* h_link, size_t link_bytes, void* d_recv,
                       size_t recv_bytes, float* d_dst, int64_t dst_elems, void* compute_stream,
                       void* copy_stream);
int zfpx_pipeline_destroy(zfpx_pipeline* pipe);

/* -------------------------------------------------------------------------
 * Variable-size modes: fixed precision and fixed accuracy
 * ---------------------------------------------------------------------- */

/*
 * ZFP's precision and accuracy modes, which the paper sets aside for future
 * work because their messages do not have a size known in advance (Sections
 * II-C and IV-B).  They run the fixed-rate block coder but stop after the
 * bit planes 31 .. 32-p of a block with exponent emax, where
 *   p = min(maxprec, max(0, emax - minexp + 8))      (8 = 2 (d+1), d = 3);
 * p = 0 codes the block as the single bit 0.
 *   precision mode: maxprec in 1..32 and minexp = ZFPX_MINEXP_NONE;
 *   accuracy mode : maxprec = 32 and minexp = zfpx_accuracy_minexp(tol):
 *                   every decoded value is within tol of its input, for
 *                   every block shorter than the cap.
 * Each block is also capped at 64*rate_cap bits (rate_cap 1..32) and cut
 * there as a fixed-rate block of that rate would be.
 *
 * Stream layout: blocks are numbered as in fixed rate (chunk order).  Block
 * b's bits, least significant first and zero padded, take nd[b] =
 * ceil(bits/32) 32-bit words (1 .. 2*rate_cap) starting at word
 * nd[0] + ... + nd[b-1].  tile_off[t] is the word offset of block 64*t for
 * t < ntiles = ceil(nblocks/64); tile_off[ntiles] is the total word count.
 * Chunk c's message is the words between the offsets of its first block and
 * of the next chunk's first block (zfpx_plan_var_chunk_offsets); its nd
 * entries rebuild every offset inside it.
 */
#define ZFPX_MINEXP_NONE (-1074)

/* minexp of accuracy mode: the largest e with 2^e <= tolerance
 * (ZFPX_MINEXP_NONE for a tolerance that is not positive). */
int zfpx_accuracy_minexp(double tolerance);

/* Sizes for a plan: the largest stream in 32-bit words (every block at the
 * cap), the tile count (tile_off has ntiles + 1 entries) and the bytes of the
 * encoder's scratch.  Any pointer may be NULL. */
int zfpx_plan_var_sizes(const zfpx_plan* plan, int rate_cap, int64_t* max_words,
                        int64_t* ntiles, size_t* work_bytes);

/*
 * Encode every chunk of the plan in a variable-size mode (one launch).
 *   d_words    : device, 4-byte aligned; words at or past words_bytes/4 are
 *                not written (the stream is then incomplete: compare
 *                tile_off[ntiles] with the capacity after synchronising; a
 *                capacity of max_words never runs out).
 *   d_nd       : device, nblocks bytes.
 *   d_tile_off : device, 8-byte aligned, ntiles + 1 entries.
 *   d_work     : device scratch of at least work_bytes (ENOSPC otherwise),
 *                4-byte aligned, contents ignored (a staging area of
 *                2*rate_cap words per block and one count per tile).  Calls
 *                that overlap in time need separate scratch.
 * Three kernels: code every tile into its staging slot, scan the tile
 * counts, copy the tiles to their offsets.
 * Errors: EINVAL for bad parameters (maxprec 1..32, minexp
 * ZFPX_MINEXP_NONE..1024, rate_cap 1..32), null or misaligned pointers or a
 * too small source.
 */
int zfpx_plan_encode_var(const zfpx_plan* plan, const float* d_src, int64_t src_elems,
                         int maxprec, int minexp, int rate_cap, uint32_t* d_words,
                         size_t words_bytes, uint8_t* d_nd, int64_t* d_tile_off, void* d_work,
                         size_t work_bytes, void* stream);

/*
 * zfpx_plan_encode_var for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same launches and results, with the staging area in a file-scope device
 * array of zfpx_noalloc_scratch_bytes() bytes (32 MiB) instead of a caller
 * workspace.  It calls no hipMalloc, hipFree or allocating routine.
 *   Limit: the plan's staging area, (2*rate_cap*nblocks + ceil(nblocks/64))
 *   32-bit words rounded up to whole 64-block tiles, must fit the array;
 *   ENOSPC otherwise (nothing enqueued).  At rate_cap 16 that is about
 *   262,000 blocks (16.7M values).
 *   Each GPU holds its own copy of the array, set up on the first call on that
 *   device (EHIP if the runtime cannot give its address) and kept until the
 *   process ends.  Every call on one GPU uses the same array and the last
 *   call's contents stay in it (nothing in it needs to start at zero): calls
 *   that overlap in time on one GPU race and give wrong streams.
 * Other arguments and errors as zfpx_plan_encode_var.
 */
int zfpx_plan_encode_var_noalloc(const zfpx_plan* plan, const float* d_src, int64_t src_elems,
                                 int maxprec, int minexp, int rate_cap, uint32_t* d_words,
                                 size_t words_bytes, uint8_t* d_nd, int64_t* d_tile_off,
                                 void* stream);
size_t zfpx_noalloc_scratch_bytes(void);

/*
 * Decode a stream made by zfpx_plan_encode_var with the same plan and
 * parameters into the plan's points of d_dst.  Any content of the words,
 * counts and offsets decodes without a fault: counts are clamped to
 * 2*rate_cap and words at or past words_bytes/4 read as zero.
 */
int zfpx_plan_decode_var(const zfpx_plan* plan, const uint32_t* d_words, size_t words_bytes,
                         const uint8_t* d_nd, const int64_t* d_tile_off, int maxprec, int minexp,
                         int rate_cap, float* d_dst, int64_t dst_elems, void* stream);

/* Word offset of each chunk's first block into d_chunk_off[0..nchunks-1] and
 * the total into d_chunk_off[nchunks] (device, 8-byte aligned): the counts
 * and displacements of an all-to-all(v) of the chunks. */
int zfpx_plan_var_chunk_offsets(const zfpx_plan* plan, const uint8_t* d_nd,
                                const int64_t* d_tile_off, int64_t* d_chunk_off, void* stream);

/* -------------------------------------------------------------------------
 * Launch configuration and autotuning
 * ---------------------------------------------------------------------- */

/*
 * A launch configuration: workgroup size in threads (64, 128 or 256; one
 * 64-block tile per wavefront) and the grid in workgroups (0 = one tile per
 * wavefront, i.e. as many workgroups as needed; otherwise a persistent grid
 * that loops over tiles).  op: 0 = pack_encode, 1 = decode_unpack.
 * zfpx_plan_set_config stores it in the plan for that op and rate (rate 0 =
 * every rate without an entry of its own); it is then used by every launch
 * on that plan.  Returns EINVAL for an unsupported configuration.  Without
 * an entry a launch uses one tile per wavefront and 128 threads, or 64 for
 * launches of more than 2^16 tiles.
 */
int zfpx_plan_set_config(zfpx_plan* plan, int op, int rate, int wg_threads, int grid_wgs);
int zfpx_plan_get_config(const zfpx_plan* plan, int op, int rate, int* wg_threads,
                         int* grid_wgs);

/*
 * Autotune: time every candidate configuration for `op` and `rate` on this
 * plan with the given buffers (the op is run repeatedly; outputs are
 * overwritten), keep the fastest in the plan and, when cache_path is not
 * NULL, record it in a small text cache keyed by device, op, rate and plan
 * shape (read first: a cached entry skips the timing).  Synchronises the
 * stream; not for hot loops.  best_us receives the chosen mean time.
 */
int zfpx_autotune(zfpx_plan* plan, int op, int rate, const float* d_src, int64_t src_elems,
                  void* d_stream_buf, size_t stream_bytes, float* d_dst, int64_t dst_elems,
                  const char* cache_path, void* stream, double* best_us);

/* -------------------------------------------------------------------------
 * Batched form captured in a HIP graph
 * ---------------------------------------------------------------------- */

/*
 * Capture, on a private stream, one pack_encode launch over every chunk of
 * the plan (d_src -> d_send) followed by one decode_unpack launch
 * (d_send -> d_dst), and instantiate the graph.  Each zfpx_graph_launch is
 * then a single hipGraphLaunch on `stream`.  Buffers are bound at creation.
 */
typedef struct zfpx_graph zfpx_graph;

int zfpx_graph_create(const zfpx_plan* plan, int rate, const float* d_src, int64_t src_elems,
                      void* d_send, size_t send_bytes, float* d_dst, int64_t dst_elems,
                      zfpx_graph** out);
int zfpx_graph_launch(zfpx_graph* graph, void* stream);
int zfpx_graph_destroy(zfpx_graph* graph);

/* -------------------------------------------------------------------------
 * Serving: continuous batching of compress / decompress requests
 * ---------------------------------------------------------------------- */

/*
 * A request codes one regular float32 array (as zfpx_encode_fixed_rate /
 * zfpx_decode_fixed_rate): op 0 compresses d_in (float32, strides sx,sy,sz)
 * into d_out (coded words, 8-byte aligned); op 1 decompresses d_in (words)
 * into d_out (float32).  Buffers are caller-owned device memory that must stay
 * valid until the request completes; the device loop runs on its own stream,
 * so work on other streams that writes them must have completed before submit.  tag is free for the caller.
 *
 * The server realises the paper's point that fixed-rate ZFP needs no
 * coordination between blocks (Section II-C) as a service: requests are
 * admitted in arrival order while a ring slot is free and their input +
 * output bytes fit in `hbm_budget_bytes`; admitted requests are cut into
 * 64-block tiles that a device-resident loop (a persistent kernel on a
 * private stream) interleaves with the tiles of every other request in
 * flight.  Results are bit-identical to the one-request launch form.
 *
 *   zfpx_server_create : max_slots ring entries (1..65536); workgroups of the
 *                        device loop (0 = 1 per compute unit; at least 2 are
 *                        launched, workgroup 0 only dispatches).  Allocates
 *                        pinned host memory and device memory.
 *   zfpx_server_submit : queue a request; EINVAL if malformed or larger than
 *                        the whole budget, EAGAIN if the host queue already
 *                        holds max_queued requests not yet admitted (the
 *                        request is not taken; submit it again later),
 *                        ESTATE once a server has taken 2^32 - 1 requests.
 *                        Thread-safe.  Returns a ticket.
 *   zfpx_server_set_max_queue : max_queued in 1 .. 2^20 (default 2^20).
 *   zfpx_server_set_idle_us : the device loop leaves after this long in which
 *                        no request was published (100 us .. 10 s, default
 *                        2000); taken at the loop's next launch.  A request
 *                        that finds the loop gone pays for a new launch
 *                        (about 15 us more on MI355X), while a running loop
 *                        holds most of every compute unit's LDS.
 *   zfpx_server_progress / _poll : collect completions and admit more;
 *                        poll reports done and the latency (seconds from
 *                        submit to the host seeing completion) and forgets
 *                        the ticket once done.
 *   zfpx_server_drain  : progress until nothing is queued or in flight
 *                        (EAGAIN after timeout_s).
 *   zfpx_server_stats  : requests admitted, largest in-flight byte total seen,
 *                        device-loop launches.
 *   zfpx_server_destroy: stop the device loop, wait for it, free.
 *   zfpx_server_replay : replay a request trace (arrival times in seconds
 *                        from the start, non-decreasing) through the server
 *                        and write each request's latency (completion minus
 *                        scheduled arrival).
 *   zfpx_plain_replay  : the same trace with one launch per request, in
 *                        arrival order on one stream (the plain form).
 */
typedef struct {
  int32_t op;
  int32_t rate;
  int64_t nx, ny, nz;
  int64_t sx, sy, sz;
  const void* d_in;
  void* d_out;
  uint64_t tag;
} zfpx_request;

typedef struct zfpx_server zfpx_server;

int zfpx_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t workgroups,
                       zfpx_server** out);
int zfpx_server_submit(zfpx_server* sv, const zfpx_request* rq, uint64_t* ticket);
int zfpx_server_progress(zfpx_server* sv);
int zfpx_server_poll(zfpx_server* sv, uint64_t ticket, int* done, double* latency_s);
int zfpx_server_drain(zfpx_server* sv, double timeout_s);
int zfpx_server_stats(zfpx_server* sv, uint64_t* admitted, size_t* max_inflight_bytes,
                      uint64_t* loop_launches);
int zfpx_server_set_max_queue(zfpx_server* sv, size_t max_queued);
int zfpx_server_set_idle_us(zfpx_server* sv, uint64_t idle_us);
int zfpx_server_destroy(zfpx_server* sv);
int zfpx_server_replay(zfpx_server* sv, const zfpx_request* rq, const double* arrival_s,
                       int64_t n, double timeout_s, double* latency_s);
int zfpx_plain_replay(const zfpx_request* rq, const double* arrival_s, int64_t n,
                      double timeout_s, void* stream, double* latency_s);

/* -------------------------------------------------------------------------
 * float16 comparator
 * ---------------------------------------------------------------------- */

/*
 * f16_truncate: d_out[i] = IEEE binary16 of d_in[i], rounded to nearest with
 * ties to even (subnormals kept, overflow to infinity, NaN stays NaN).
 * f16_restore: exact widening back to float32.  The paper's comparator casts
 * the buffer to float16 before sending and back on receipt (Sections I and
 * IV-F).  n may be 0; pointers must be 4-byte (in) / 2-byte (out) aligned.
 */
int f16_truncate(const float* d_in, size_t n, uint16_t* d_out, void* stream);
int f16_restore(const uint16_t* d_in, size_t n, float* d_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ZFPX_H */
