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
struct PlanEntry {
  uint32_t block;
  uint32_t seq_base;  // first token slot of this block in the token scratch
  uint64_t dst;
};

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
  uint8_t* lit;    // token scratch: n_plan * B literal bytes
  uint8_t* lens;   // 4 bytes per sequence
  uint8_t* offs;   // ow bytes per sequence
  uint32_t* err;   // sticky error word
  unsigned long long* ext_bytes;  // counter: match bytes read from earlier blocks
  // persistent-kernel state
  uint32_t* queue;      // work counter
  uint32_t* done;       // per-block completion epochs
  uint32_t epoch;
  uint64_t wait_ticks;  // bound of one dependency wait, in 100 MHz clock ticks
};

// Kernel launchers (kernels.hip).  All asynchronous on `s`.
hipError_t launch_rans(const DecodeArgs& a, hipStream_t s);
hipError_t launch_expand_level(const DecodeArgs& a, uint32_t plan_lo, uint32_t plan_hi,
                               hipStream_t s);
hipError_t launch_persistent(const DecodeArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_copy(const DecodeArgs& a, const CopyItem* items, uint32_t n_items,
                       hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);

}  // namespace ace
