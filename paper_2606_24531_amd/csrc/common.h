// Internal structures shared by the host planner (host.cpp) and the gfx950
// kernels (kernels.hip) of libaceseek.  Nothing here is part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ace {

// Archive layout constants (the byte format both readers of an archive
// agree on; this library parses it with its own code).
constexpr uint32_t kMagic = 0x314B5341u;  // "ASK1"
constexpr uint32_t kHdr = 64, kBlk = 32, kSDesc = 16;
constexpr uint32_t kProbBits = 12, kM = 4096, kL = 65536;

// Device error word bits (sticky in the workspace header).
constexpr uint32_t kErrCorrupt = 1u, kErrTimeout = 2u;

// One block to decode in a call.  dst is where the block's first byte goes,
// relative to DecodeArgs::dst_base.
// One planned block, with the index fields its kernels need, so that a
// kernel reaches the block's tokens with one load of its plan entry.
struct PlanEntry {
  uint32_t block;
  uint32_t seq_base;  // first token slot of this block in the token scratch
  uint64_t dst;       // where the block's bytes go (added to dst_base)
  uint64_t pay;       // offset of the block payload in the archive
  uint32_t n_seq, n_lit, dep_off, dep_cnt;
  uint64_t raw[3];    // archive offset of the LIT, LEN, OFF data when stored raw, else kCoded
};
static_assert(sizeof(PlanEntry) == 64, "plan entries are 64 bytes");
constexpr uint64_t kCoded = ~0ull;

// One contiguous copy of decoded bytes: [src_abs, src_abs + len) of the
// decompressed coordinate space into dst (device address).  Blocks are
// found through the location table.
struct CopyItem {
  uint64_t src_abs;
  uint64_t dst;
  uint32_t len;
  uint32_t pad;
};

struct DecodeArgs {
  const uint8_t* arch;  // device archive (with ACE_ARCH_PAD slack)
  const PlanEntry* plan;
  uint32_t n_plan;
  uint32_t B, W, ow, n_blocks;
  uint64_t n_total;
  uint64_t dst_base;
  uint64_t* loc;   // block id -> device address of its decoded bytes
  uint32_t loc_linear;  // 1: block b lives at dst_base + b * B (whole-archive decode)
  uint32_t b_shift;     // log2(B) when B is a power of two, else 64
  uint8_t* lit;    // token scratch: n_plan * B literal bytes
  uint8_t* lens;   // 4 bytes per sequence
  uint8_t* offs;   // ow bytes per sequence
  uint32_t* err;   // sticky error word
  unsigned long long* ext_bytes;  // counter: match bytes read from earlier blocks
  // persistent-kernel state
  uint32_t n_lvl;       // dependency levels of the plan (bounds in lvl_dev)
  uint32_t* lvl_done;   // per level: expansions finished and published
  uint32_t* lvl_claim;  // per slice and level: expansions claimed (slice-major rows)
  uint32_t lvl_row;     // words per slice row of lvl_claim
  uint32_t* lvl_seen;   // levels finished, in copies one 128-byte line apart
  // per level and XCD: blocks done so far << 32 | workgroups expanding, then
  // the blocks already written back (kMaxXcc of each per level)
  unsigned long long* lvl_xcd;
  uint32_t max_polls;   // consecutive idle polls before a wait gives up
  // plan length (device-planned batches; null for host-planned calls) and
  // level boundaries in device memory (device-planned batches and the
  // persistent kernel)
  const uint32_t* n_plan_dev;
  const uint32_t* lvl_dev;
  // per-block clock trace (null: off): eight u64 per plan entry, the 100 MHz
  // device clock at the start and end of its expansion and of each of its
  // three entropy streams
  unsigned long long* trace;
};

// Entropy coding of token streams on the device (the encoder's rANS step):
// stream i has n[i] symbols at sym + sym_off[i]; its coded form (table,
// W states, words) is written at out + out_off[i] (capacity 544 + 4 W +
// 2 n[i]), its byte count to out_len[i] (0: the stream stays raw), with
// scratch + scr_off[i] (2 n[i] bytes) for the words.  policy: 0 rANS when
// smaller than raw, 1 always rANS, 2 always raw.
struct EncArgs {
  const uint8_t* sym;
  const uint64_t* sym_off;
  const uint32_t* n;
  uint8_t* out;
  const uint64_t* out_off;
  uint16_t* scratch;
  const uint64_t* scr_off;
  uint32_t* out_len;
  uint32_t W, policy, n_streams;
};
hipError_t launch_rans_encode(const EncArgs& e, hipStream_t s);

// Device-side planning of a batch of seeks (captured once in a HIP graph).
// Per call, `desc` holds: u64 n, u64 d_out, then n x (lo, hi, out_off).
struct BatchArgs {
  const uint8_t* arch;
  uint32_t B, n_blocks, depth, cap;
  uint64_t n_total;
  const uint32_t* order;   // all blocks by level (static)
  const uint32_t* lstart;  // level boundaries in `order` (depth + 1, static)
  uint8_t* need;           // per block: needed by this batch
  uint32_t* pre;           // per position in `order`: needed blocks before it
  const uint64_t* desc;
  PlanEntry* plan;
  uint32_t* n_plan_dev;
  uint32_t* lvl_dev;       // depth + 1 plan boundaries per level
  uint64_t* loc;
  const uint8_t* pin;        // per block: 1 = decoded once and kept (its loc stays valid)
  const uint32_t* pin_base;  // slots taken by kept blocks; planned blocks go after them
  uint32_t* chunk_cnt;       // compaction: per chunk of `order`, needed blocks (then their prefix)
  uint32_t* chunk_seq;       // and their sequences; batch_compact_chunks + 1 entries each
};

// Kernel launchers (kernels.hip).  All asynchronous on `s`.
// per_wave: streams one wavefront decodes (0 = 2 when W <= 32, else 1);
// waves: wavefronts per block in the expansion (1, 2, 4 or 8; 0 = 4 while
// the launch's blocks fit on the device at once as four-wavefront
// workgroups, else 2)
hipError_t launch_rans(const DecodeArgs& a, uint32_t lo, uint32_t hi, uint32_t per_wave, hipStream_t s);
hipError_t launch_expand_level(const DecodeArgs& a, uint32_t plan_lo, uint32_t plan_hi, uint32_t waves,
                               hipStream_t s);
// the persistent level-by-level expansion (kernel (c)); grid 0 = as many
// workgroups as the device holds at once.  Its counters (persist_sync_words
// words from lvl_done, laid out by persist_sync) start at zero.
constexpr uint32_t kPersistSlices = 8, kPersistReplicas = 64, kPersistLine = 32, kMaxXcc = 16;
inline uint64_t persist_row(uint32_t n_lvl) { return (n_lvl + kPersistLine - 1ull) / kPersistLine * kPersistLine; }
inline uint64_t persist_sync_words(uint32_t n_lvl) {
  return (1 + kPersistSlices) * persist_row(n_lvl) + (uint64_t)kPersistReplicas * kPersistLine +
         4ull * kMaxXcc * n_lvl;
}
// Points the kernel's counters into `words` (128-byte aligned, at least
// persist_sync_words(a.n_lvl) words): finished counts, one row per level;
// claim counts, one row per slice; the finished-level copies; per level,
// 2 kMaxXcc 64-bit counters (two per XCD).
inline void persist_sync(DecodeArgs& a, uint32_t* words) {
  const uint64_t row = persist_row(a.n_lvl);
  a.lvl_done = words;
  a.lvl_claim = words + row;
  a.lvl_row = (uint32_t)row;
  a.lvl_seen = words + (1 + kPersistSlices) * row;
  a.lvl_xcd = reinterpret_cast<unsigned long long*>(a.lvl_seen + (uint64_t)kPersistReplicas * kPersistLine);
}
hipError_t launch_persistent(const DecodeArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_copy(const DecodeArgs& a, const CopyItem* items, uint32_t n_items,
                       hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
// The fixed device scratch of the allocation-free seek (kStaticScratchBytes,
// one copy per device): this device's address of it.
constexpr uint64_t kStaticScratchBytes = 64ull << 20;
hipError_t static_scratch(void** ptr);
// batch planning and gather (device-side counts; grids sized for capacity)
hipError_t launch_batch_mark(const BatchArgs& b, hipStream_t s);
hipError_t launch_batch_close(const BatchArgs& b, uint32_t level, uint32_t width, hipStream_t s);
hipError_t launch_batch_compact(const BatchArgs& b, hipStream_t s);
uint32_t batch_compact_chunks(uint32_t n_blocks);
hipError_t launch_batch_gather(const BatchArgs& b, const DecodeArgs& a, hipStream_t s);
// a one-request descriptor (n = 1, d_out, then lo, hi at output offset 0)
// written by a kernel from its arguments
hipError_t launch_put_range(uint64_t* desc, uint64_t d_out, uint64_t lo, uint64_t hi, hipStream_t s);
hipError_t launch_rans_dev(const DecodeArgs& a, uint32_t cap, uint32_t per_wave, hipStream_t s);
// entropy decode of levels [lv_lo, lv_hi), whose plan range is read from
// lvl_dev; width = the most entries those levels can hold
hipError_t launch_rans_levels_dev(const DecodeArgs& a, uint32_t lv_lo, uint32_t lv_hi, uint32_t width,
                                  uint32_t per_wave, hipStream_t s);
// queries (once per device) what the automatic expansion shape needs; call
// before a stream capture that launches expansions
hipError_t prepare_expand_shapes();
hipError_t launch_expand_level_dev(const DecodeArgs& a, uint32_t level, uint32_t width, uint32_t waves,
                                   hipStream_t s);

}  // namespace ace
