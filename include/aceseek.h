/*
 * aceseek.h -- C ABI of libaceseek, a gfx950 (MI355X) decoder for archives
 * of the two-layer absolute-offset codec: per-block interleaved rANS over
 * three token streams (literals, lengths, absolute offsets), then an LZ77
 * match layer whose back-references name absolute positions in the output.
 *
 * The paper's central operation is a seek: decode one absolute byte range
 * through both layers, in isolation (Sections 3 and 5).  Section 2 gives the
 * reason it is possible: offsets are absolute, so a block can be decoded as
 * soon as the earlier blocks its matches copy from are decoded, however the
 * decoder reached it.
 * Section 7 adds range decoding of many blocks.
 *
 * Conventions
 *  - Every function returns ACE_OK (0) or a negative ACE_E_* code and, on
 *    error, leaves a description for ace_last_error() (per thread).
 *  - Pointers named d_* are device (HBM) pointers, h_* are host pointers.
 *    The caller owns every buffer; the library never allocates or frees
 *    device memory (the one exception is the fixed scratch of
 *    ace_seek_static, a static device array of the loaded library).  An
 *    ace_archive owns only a host copy of the index.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Device work is
 *    asynchronous on it; host-side validation errors are returned at once,
 *    device-side ones (corrupt token streams) are sticky in the workspace
 *    and read by ace_check().
 *  - Calls on different streams must use different workspaces.  A fresh
 *    workspace's first 256 bytes must be zero (its error word and counters);
 *    ace_check() and ace_read_counters() clear what they read.
 */
#ifndef ACESEEK_H
#define ACESEEK_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ACE_OK 0
#define ACE_E_ARG (-1)     /* null pointer, bad parameter, lo > hi */
#define ACE_E_RANGE (-2)   /* range beyond the decompressed size */
#define ACE_E_CORRUPT (-3) /* archive fails validation */
#define ACE_E_NOSPACE (-4) /* output or workspace too small */
#define ACE_E_HIP (-5)     /* HIP runtime error */
#define ACE_E_TIMEOUT (-6) /* a bounded device wait expired */
#define ACE_E_NOMEM (-7)   /* host allocation failed */

/* Bytes of readable slack the device copy of an archive must have after its
 * last byte (kernels stage stream data in 16-byte-aligned chunks). */
#define ACE_ARCH_PAD 4096u

/* Encoder parameters.  None of them affects how an archive decodes.
 *  block_size  B, bytes per block, 1 .. 2^24
 *  interleave  W, rANS states per stream, 1 .. 64
 *  min_match   shortest match emitted (>= hash_len)
 *  hash_len    bytes hashed per position, 1 .. 64
 *  max_chain   hash-chain candidates examined per position
 *  max_level   0 = unbounded; else every block's dependency level < max_level
 *  flags       bits 0-1, stream-mode policy: 0 = rANS only where smaller,
 *              1 = always rANS, 2 = always raw; bit 2 (ACE_ENC_WIDE_OFFSETS):
 *              store absolute offsets in 8 bytes even when every position
 *              fits in 4 (the width archives above 4 GiB need); bit 3
 *              (ACE_ENC_DEVICE_ENTROPY): the rANS step of every stream runs
 *              on the current device (one wavefront per stream, the same
 *              archive bytes as the host's; the parse stays on the host;
 *              device memory is allocated and freed within the call, and a
 *              HIP failure returns ACE_E_HIP); other bits are ACE_E_ARG
 *  n_threads   host threads for the parse (0 = all cores) */
#define ACE_ENC_WIDE_OFFSETS 4u
#define ACE_ENC_DEVICE_ENTROPY 8u
typedef struct {
  uint32_t block_size, interleave, min_match, hash_len, max_chain, max_level, flags, n_threads;
} ace_encode_params;

/* A half-open range [lo, hi) of absolute positions in the decompressed data. */
typedef struct {
  uint64_t lo, hi;
} ace_range;

/* Launch shape.  Zero fields take the library defaults; a value the library
 * does not offer is ACE_E_ARG.
 *  waves_per_block  wavefronts cooperating on one block's match expansion:
 *                   1, 2, 4 or 8; each takes two sequences per lane per
 *                   tile.  0 = per launch: 4 while the launch's blocks fit
 *                   on the device at once as four-wavefront workgroups
 *                   (then one block's latency sets the time), else 2 (more
 *                   blocks in flight)
 *  blocks_per_wg    blocks whose streams one entropy wavefront decodes side
 *                   by side: 1, or 2 when the interleave is at most 32
 *                   (0 = 2 when possible)
 *  lut_variant      entropy table layout in LDS: 0 = 4096-byte slot->symbol
 *                   map plus one (f-1, cum) word per symbol (the only one)
 *  grid_wgs         workgroups of the persistent expansion (0 = as many as
 *                   the device holds at once; never more than the planned
 *                   blocks)
 *  mode             0 and 1: one entropy launch for every planned block,
 *                   then one match-expansion launch per dependency level,
 *                   all on the caller's stream; 2: one entropy launch,
 *                   then one persistent launch that expands every level in
 *                   turn, synchronised by counters in the workspace (every
 *                   wait bounded by a count of idle polls: an expired wait
 *                   makes ace_check report ACE_E_TIMEOUT, and the launch
 *                   still ends); 3: the levels split in an early
 *                   group (at most a quarter of the planned blocks, at
 *                   least level 0) and a late group; the late group's
 *                   entropy decode runs as one launch on a second stream of
 *                   the calling thread (created on first use, one per
 *                   device) while the caller's stream decodes and expands
 *                   the early group, then waits for it and expands the late
 *                   levels (so the caller's stream is joined with the
 *                   second stream before the call's last launch) */
typedef struct {
  uint32_t waves_per_block, blocks_per_wg, lut_variant, grid_wgs, mode;
} ace_tuning;

typedef struct ace_archive ace_archive;

const char* ace_last_error(void);

/* ---- host encoder (the paper's encoder runs on the CPU, Section 2) ---- */
/* Upper bound on the archive size for n input bytes. */
int ace_encode_bound(uint64_t n, const ace_encode_params* p, uint64_t* bound);
/* Encodes h_src[0..n) into h_dst (capacity dst_cap); *dst_len receives the
 * archive size (also when ACE_E_NOSPACE is returned). */
int ace_encode_archive(const uint8_t* h_src, uint64_t n, const ace_encode_params* p,
                       uint8_t* h_dst, uint64_t dst_cap, uint64_t* dst_len);

/* ---- archive residency (Section 9: data stays compressed-resident) ----
 * h_arch: the archive bytes in host memory (read during the call only);
 * d_arch: the same bytes already copied to the device, with ACE_ARCH_PAD
 * readable bytes after them, kept alive by the caller while the handle is
 * used.  Validates the header, block table, dependency lists, levels and
 * stream descriptors; token-level checks happen on the device. */
int ace_archive_open(const uint8_t* h_arch, uint64_t len, const void* d_arch, ace_archive** out);
void ace_archive_close(ace_archive* a);
int ace_archive_info(const ace_archive* a, uint64_t* n_total, uint32_t* block_size,
                     uint32_t* n_blocks, uint32_t* depth);

/* ---- out-of-core range decode (Section 7: when the archive is larger than
 * device memory, ranges are decoded with only the blocks they need on the
 * device) ----
 * ace_archive_open_ooc: validates the archive in host memory as
 * ace_archive_open does and keeps h_arch (caller-owned, unchanged and alive
 * while the handle is used); nothing is uploaded.  Such a handle is taken by
 * ace_seek_ooc, ace_seek_ooc_bytes, ace_archive_info and ace_archive_close;
 * the calls that read a resident archive return ACE_E_ARG for it.
 * ace_seek_ooc_bytes: the workspace ace_seek_ooc needs for [lo, hi) (0 for
 * an empty range): the host-planned seek's, plus the staged dependency lists
 * and payloads of the range's dependency closure, plus ACE_ARCH_PAD.
 * ace_seek_ooc: writes exactly hi - lo bytes at d_out (device).  The host
 * plans the closure, copies the planned blocks' dependency lists and
 * payloads from h_arch into d_ws (device, ws_cap bytes) through a pinned
 * staging buffer held by the handle, and the same kernels as ace_seek decode
 * them there.  Returns once the work has finished on `stream` (calls on one
 * handle take turns on its staging buffer).  Errors: ACE_E_ARG (a handle
 * not opened out of core, null pointers), ACE_E_RANGE, ACE_E_NOSPACE (the
 * needed size is in the message); the device's error word is read with
 * ace_check(d_ws, stream) as after ace_seek. */
int ace_archive_open_ooc(const uint8_t* h_arch, uint64_t len, ace_archive** out);
int ace_seek_ooc_bytes(const ace_archive* a, uint64_t lo, uint64_t hi, uint64_t* bytes);
int ace_seek_ooc(const ace_archive* a, uint64_t lo, uint64_t hi, uint8_t* d_out, void* d_ws,
                 uint64_t ws_cap, const ace_tuning* t, void* stream);

/* Optional: the whole-archive decode plan (the blocks in dependency-level
 * order with the index fields the kernels need, 64 bytes per block, then the
 * block ids in that order and the level boundaries) kept resident on the
 * device.  ace_plan_bytes gives its size; attach uploads it once into d_plan
 * (caller-owned device memory of at least that many bytes, kept alive and
 * unmodified while the handle is used; synchronous on `stream`).  Later
 * ace_decode_all calls read it there instead of copying it from the host on
 * every call, and ace_seek can plan on the device. */
int ace_plan_bytes(const ace_archive* a, uint64_t* bytes);
int ace_archive_attach_plan(ace_archive* a, void* d_plan, uint64_t bytes, void* stream);

/* Workspace bytes needed to decode the given ranges (ranges == NULL and
 * n_ranges == 0: the whole archive): the plan, the location table, token
 * scratch and the slots of blocks decoded only as sources of the ranges'
 * dependency closure (Section 2: the blocks a range needs are the targets
 * and, recursively, the earlier blocks their matches copy from). */
int ace_workspace_bytes(const ace_archive* a, const ace_range* ranges, uint32_t n_ranges,
                        uint64_t* bytes);

/* An upper bound of ace_workspace_bytes over every set of at most n_ranges
 * ranges whose lengths add up to at most total_bytes (every block in the
 * closure and decoded into a slot), so that a caller can allocate one
 * workspace before any request is known. */
int ace_workspace_bound(const ace_archive* a, uint32_t n_ranges, uint64_t total_bytes,
                        uint64_t* bytes);

/* Whole-archive decode (Section 2: every block, both layers, each after the
 * earlier blocks it copies from; Section 7: decode of a whole block range):
 * writes n_total bytes at d_out (out_cap >= n_total).  The workspace needs
 * ace_workspace_bytes(a, NULL, 0) bytes. */
int ace_decode_all(const ace_archive* a, uint8_t* d_out, uint64_t out_cap, void* d_ws,
                   uint64_t ws_cap, const ace_tuning* t, void* stream);

/* Seek (Section 5): writes exactly hi - lo bytes at d_out and nothing else in
 * d_out.  Blocks that only supply sources are decoded into the workspace.
 * An empty range returns ACE_OK without launching.  Planning: when the
 * archive's plan is attached (ace_archive_attach_plan) and ws_cap is at
 * least ace_batch_workspace_bytes(a, 1), the range's dependency closure is
 * found on the device (the batch planner's kernels for one request) and the
 * host only enqueues; otherwise the host walks the closure, and the
 * workspace needs ace_workspace_bytes for the range.  Both give the same
 * bytes. */
int ace_seek(const ace_archive* a, uint64_t lo, uint64_t hi, uint8_t* d_out, void* d_ws,
             uint64_t ws_cap, const ace_tuning* t, void* stream);

/* Allocation-free seek, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same result as ace_seek, with the workspace taken from a
 * fixed device scratch inside the library (ACE_STATIC_SCRATCH_BYTES, one copy
 * per device, held until the process ends) instead of a caller buffer.  The
 * call allocates nothing: no hipMalloc, hipFree or allocating library call.
 * d_status (caller-owned device memory, 4 bytes) receives the device error
 * word of this seek once it completes on `stream` (0 = ok; bit 0 = a token
 * stream broke a format rule, bit 1 = a bounded dependency wait expired).
 * Runs the per-level path: t may be NULL or ask for mode 0 or 1, and phase
 * timing must be off (ACE_E_ARG otherwise).  A seek whose workspace would
 * exceed the scratch fails with ACE_E_NOSPACE (the needed size is in the
 * message).  Every call on one device shares that device's scratch and the
 * scratch keeps the last call's contents: calls that overlap on one device
 * (two host threads, or two streams not ordered by the caller) race and may
 * return wrong bytes; order them on one stream. */
#define ACE_STATIC_SCRATCH_BYTES (64ull << 20)
int ace_seek_static(const ace_archive* a, uint64_t lo, uint64_t hi, uint8_t* d_out, uint32_t* d_status,
                    const ace_tuning* t, void* stream);

/* Batched seek: many seeks of Section 5 served together (Section 7: range
 * decode of many blocks at once).  Request i writes [lo_i, hi_i) at d_out +
 * h_out_off[i] (host arrays; the output ranges must not overlap).  All
 * requests share one dependency-ordered decode of the union of their
 * closures, then one gather.  Errors as for ace_seek. */
int ace_seek_batch(const ace_archive* a, const ace_range* h_ranges, uint32_t n,
                   uint8_t* d_out, const uint64_t* h_out_off, void* d_ws, uint64_t ws_cap,
                   const ace_tuning* t, void* stream);

/* Waits for the stream, reads and clears the workspace's sticky device error
 * word: ACE_OK, ACE_E_CORRUPT (a token stream broke one of the format rules
 * of Section 2's token grammar as this library reads it) or ACE_E_TIMEOUT (a
 * bounded dependency wait expired). */
int ace_check(void* d_ws, void* stream);

/* ---- batched seek as one replayed HIP graph ----
 * A batch context owns a HIP graph captured once on `stream`.  Each run
 * uploads the request descriptors (one small host-to-device copy) and
 * replays the graph: device-side planning (targets of every request, their
 * dependency closure, a level-ordered plan), the decode of the union into
 * workspace slots (one entropy launch, one expansion launch per level), and
 * a gather of every request to its output offset.  Capacity is fixed at creation; counts are read on the device, so
 * any batch up to the capacity replays the same graph.  The workspace must
 * stay dedicated to the context.  Runs are asynchronous on the stream; a run
 * waits for the previous run of the same context to have started reading its
 * descriptors.  Errors are read with ace_check(d_ws, stream). */
typedef struct ace_batch ace_batch;
int ace_batch_workspace_bytes(const ace_archive* a, uint32_t max_requests, uint64_t* bytes);
int ace_batch_create(const ace_archive* a, uint32_t max_requests, void* d_ws, uint64_t ws_cap,
                     const ace_tuning* t, void* stream, ace_batch** out);
/* Request i writes [lo_i, hi_i) at d_out + h_out_off[i]. */
int ace_batch_run(ace_batch* b, const ace_range* h_ranges, uint32_t n, uint8_t* d_out,
                  const uint64_t* h_out_off);
/* Decoded-block cache for serving.  The archive stays compressed-resident
 * (Section 9), but every seek's closure reaches down to the lowest
 * dependency levels, and a range decode is latency-bound (Section 7).  This
 * call decodes every block of levels [0, levels) once, into the first slots
 * of the batch's workspace, and keeps them: later runs neither plan nor
 * decode those blocks (their closures stop there) and read them in place.
 * Costs no extra memory (the workspace already has a slot per block).
 * Synchronous on the batch's stream (it waits for a pending run first).
 * Once per context: a second call is ACE_E_ARG; levels above the archive's
 * depth are ACE_E_ARG; 0 keeps nothing.  ACE_E_CORRUPT if the decode of the
 * kept levels failed (their blocks are then not kept). */
int ace_batch_pin(ace_batch* b, uint32_t levels);
void ace_batch_destroy(ace_batch* b);

/* Waits for the stream, then reads and clears the workspace's counter of
 * match bytes that were copied from earlier blocks (the external source
 * bytes of every decode since the last read).  With the archive size and the
 * output size this gives the algorithmic HBM bytes of a decode. */
int ace_read_counters(void* d_ws, void* stream, uint64_t* ext_src_bytes);

/* Phase timing for measurement: with timing on, every decode on the calling
 * thread records HIP events on its stream before and after the entropy
 * launch and after the last match-expansion launch (no work is skipped).
 * ace_last_timings waits for the last timed decode and returns the two
 * phases' durations in milliseconds. */
int ace_set_timing(int on);

/* Per-block clock trace for measurement.  While d_trace is set (device
 * memory of `bytes` bytes; null turns the trace off), each whole-archive
 * decode or seek issued by the calling thread records, per planned block i
 * (plan order = level order), eight u64 values of the device's 100 MHz
 * constant clock at d_trace[8 i ...]: the start and end of the block's match
 * expansion, then start and end of its LIT, LEN and OFF entropy decode (left
 * untouched for streams stored raw).  A decode that plans more blocks than
 * bytes / 64 fails with ACE_E_NOSPACE.  The caller owns the buffer. */
int ace_set_block_trace(void* d_trace, uint64_t bytes);
int ace_last_timings(float* ms_entropy, float* ms_match);

/* Host time of the last timed decode or seek on the calling thread (phase
 * timing on), in microseconds: planning (from the call's entry to its first
 * enqueue: range closure, level order, plan entries, workspace layout) and
 * enqueueing (plan upload and launches; the device work is not waited for).
 * ACE_E_ARG when no timed call has run on this thread. */
int ace_last_host_times(double* us_plan, double* us_enqueue);

#ifdef __cplusplus
}
#endif
#endif
