// gfx950 kernels of libaceseek: two-layer decode of absolute-offset LZ77
// archives (entropy layer: interleaved rANS; match layer: absolute-offset
// copies).  Paper Sections 2, 3 and 5; the rANS is Duda's, interleaved as in
// Giesen's construction (paper Section 9 cites both lines of work).
//
// Wave64 everywhere.  No MFMA: the path is integer decode and byte movement.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <mutex>
#include <type_traits>

#include "common.h"

namespace ace {
namespace {


// Device memory seen through the global address space.  Loads and stores
// through these pointers are global instructions, which count only against
// the vector-memory counter; through a generic pointer they are flat
// instructions, which also count against the LDS counter, so that a wait for
// an LDS result would also wait for every load and store still in flight.
#ifndef ACE_GLOBAL
#define ACE_GLOBAL __attribute__((address_space(1)))
#endif
// An empty asm that makes the compiler treat x as changed (keeps a value
// computed for every lane instead of under a branch).
#ifndef ACE_OPAQUE
#define ACE_OPAQUE(x) __asm__ volatile("" : "+v"(x))
#endif
template <typename T>
__device__ __forceinline__ ACE_GLOBAL T* gp(T* p) {
  return (ACE_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ const ACE_GLOBAL T* gp(const T* p) {
  return (const ACE_GLOBAL T*)p;
}
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint8_t ld8(const uint8_t* p) { return *gp(p); }
__device__ __forceinline__ void st8(uint8_t* p, uint8_t v) { *gp(p) = v; }
__device__ __forceinline__ void st16(uint8_t* p, uint4 v) {  // 16-aligned p
  u32x4 w;
  w.x = v.x;
  w.y = v.y;
  w.z = v.z;
  w.w = v.w;
  *gp(reinterpret_cast<u32x4*>(p)) = w;
}

__device__ __forceinline__ uint32_t ld16(const uint8_t* p) {
  return (uint32_t)ld8(p) | ((uint32_t)ld8(p + 1) << 8);
}
__device__ __forceinline__ uint32_t ld32(const uint8_t* p) {
  return *gp(reinterpret_cast<const uint32_t*>(p));  // callers pass 4-aligned addresses
}
__device__ __forceinline__ uint64_t ld64(const uint8_t* p) {
  return (uint64_t)ld32(p) | ((uint64_t)ld32(p + 4) << 32);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}


// Lane-shifted copy of v for an inclusive scan (DPP, no LDS): kCtl selects
// the source lane (row_shr:n = 0x110 + n within rows of 16 lanes; 0x142 =
// row_bcast:15, the last lane of each row into the next row; 0x143 =
// row_bcast:31, lane 31 into rows 2 and 3) and kRows the rows written.
// Lanes without a source, or in rows not written, read 0: the identity of
// both sum and max over unsigned values.
template <int kCtl, int kRows>
__device__ __forceinline__ uint32_t dpp_src(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kCtl, kRows, 0xf, false);
}

// Inclusive scan over aligned groups of G lanes (G = 32 or 64) under op (a
// sum or a max): shifts by 1, 2, 4 and 8 within each row, then row 0's and
// row 2's last lanes into rows 1 and 3; for G = 64 also lane 31 into rows 2
// and 3.  Every lane of the wavefront must be active.
template <uint32_t G, typename Op>
__device__ __forceinline__ uint32_t grp_scan(uint32_t v, Op op) {
  static_assert(G == 32 || G == 64, "groups of 32 or 64 lanes");
  v = op(v, dpp_src<0x111, 0xf>(v));
  v = op(v, dpp_src<0x112, 0xf>(v));
  v = op(v, dpp_src<0x114, 0xf>(v));
  v = op(v, dpp_src<0x118, 0xf>(v));
  v = op(v, dpp_src<0x142, 0xa>(v));
  if (G == 64) v = op(v, dpp_src<0x143, 0xc>(v));
  return v;
}
struct OpAdd {
  __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a + b; }
};
struct OpMax {
  __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a > b ? a : b; }
};

__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v, uint32_t) { return grp_scan<64>(v, OpAdd{}); }
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t v) { return grp_scan<64>(v, OpMax{}); }
// the value of lane 63 (uniform)
__device__ __forceinline__ uint32_t lane63(uint32_t v) { return (uint32_t)__builtin_amdgcn_readlane((int)v, 63); }
__device__ __forceinline__ uint32_t wave_total(uint32_t v) { return lane63(wave_incl_sum(v, 0)); }

__device__ __forceinline__ void flag(uint32_t* err, uint32_t bit) { atomicOr(err, bit); }

// Block index of absolute position x (a shift for power-of-two block sizes).
__device__ __forceinline__ uint64_t blk_of(const DecodeArgs& a, uint64_t x) {
  return a.b_shift < 64 ? x >> a.b_shift : x / a.B;
}

// ---------------------------------------------------------------------------
// Entropy layer: a group of G lanes (G = 64, or 32 when W <= 32, so that one
// wavefront decodes two streams side by side) decodes one rANS stream.
//
// LDS holds each stream's 12-bit table as a 4096-byte slot -> symbol map plus
// one packed word per symbol (f << 16 | cum), and a ring of two chunks of
// renormalisation words (8 G bytes each), refilled from a register
// prefetch so the decode loop never waits on HBM latency.  The table build's
// scratch lives in the ring before the ring is filled.  Lane j of a group
// owns state j; each step decodes symbols t*W .. t*W+W-1, and the lanes that
// renormalise take consecutive words in lane order: word = running position
// + (count of renormalising lanes below in the group).  The loop body is
// branch-free apart from the ring refill, and each step's symbols are stored
// straight to the output (one coalesced store per step, no LDS staging).
// ---------------------------------------------------------------------------
template <uint32_t G>
struct RansGroup {
  uint8_t sym[4096];  // slot -> symbol
  uint32_t fc[256];   // symbol -> f << 16 | cum
  union {
    u32x2 ring[2 * G];  // 2 chunks x G lanes x 8 B
    struct {
      unsigned long long starts[64];  // bit t set: a symbol's interval starts at slot t
      uint8_t by_rank[256];           // k-th present symbol
    } b;
  } u;
};

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Inclusive prefix sum over aligned groups of G lanes, and the group's
// total read from its last lane (group h = lane / G).
template <uint32_t G>
__device__ __forceinline__ uint32_t grp_incl_sum(uint32_t v) { return grp_scan<G>(v, OpAdd{}); }
template <uint32_t G>
__device__ __forceinline__ uint32_t grp_last(uint32_t incl, uint32_t h) {
  if (G == 64) return lane63(incl);
  const uint32_t t0 = (uint32_t)__builtin_amdgcn_readlane((int)incl, 31), t1 = lane63(incl);
  return h ? t1 : t0;
}

// Whether any lane of group h has v set.
template <uint32_t G>
__device__ __forceinline__ bool grp_any(bool v, uint32_t h) {
  const uint64_t m = __ballot(v);
  return G == 64 ? m != 0 : ((m >> (32 * h)) & 0xFFFFFFFFull) != 0;
}

// Decodes one stream per group; `on` (group-uniform) says whether the group
// has a stream.  Every lane of the wave must call it.  Returns true (for the
// group's lanes) when the group's stream breaks a format rule.
template <uint32_t G>
__device__ __forceinline__ bool rans_decode_group(const uint8_t* src, uint32_t clen, uint32_t n, uint32_t W,
                                                  uint8_t* dst, RansGroup<G>& sm, uint32_t g, uint32_t h,
                                                  bool on) {
  constexpr uint32_t kSpl = 256 / G;      // symbols per lane in the table build
  constexpr uint32_t kChunkW = 4 * G;     // words per ring chunk (at least the kU * W of one check)
  // ---- frequency table: 32-byte presence bitmap, then f-1 per present symbol
  bool bad = on && clen < 32;
  on = on && !bad;
  const uint32_t bits = !on ? 0u
                        : G == 64 ? ((uint32_t)src[g >> 1] >> ((g & 1) * 4)) & 0xFu
                                  : (uint32_t)src[g];
  const uint32_t cnt = __popc(bits);
  const uint32_t cnt_in = grp_incl_sum<G>(cnt);
  const uint32_t before = cnt_in - cnt;
  const uint32_t present = grp_last<G>(cnt_in, h);
  const uint32_t tsz = (32 + 2 * present + 3) & ~3u;
  if (on && (present == 0 || tsz + 4 * W > clen || ((clen - tsz - 4 * W) & 1))) bad = true;
  on = on && !bad;
  uint32_t f[kSpl], mysum = 0, k = before;
#pragma unroll
  for (uint32_t j = 0; j < kSpl; j++) {
    f[j] = (on && ((bits >> j) & 1)) ? ld16(src + 32 + 2 * (k++)) + 1 : 0;
    mysum += f[j];
  }
  const uint32_t sum_in = grp_incl_sum<G>(mysum);
  uint32_t cum = sum_in - mysum;
  const uint32_t total = grp_last<G>(sum_in, h);
  if (on && total != kM) bad = true;
  on = on && !bad;
  for (uint32_t j = g; j < 64; j += G) sm.u.b.starts[j] = 0ull;
  wave_sync();
  k = before;
  if (on) {
#pragma unroll
    for (uint32_t j = 0; j < kSpl; j++) {
      const uint32_t s = kSpl * g + j;
      sm.fc[s] = f[j] ? (f[j] << 16) | cum : 0u;
      if (f[j]) {
        sm.u.b.by_rank[k++] = (uint8_t)s;
        atomicOr(&sm.u.b.starts[cum >> 6], 1ull << (cum & 63));
      }
      cum += f[j];
    }
  }
  wave_sync();
  // ---- slot -> symbol: lane g fills slots 4096/G * g onwards in order, the
  // rank of the covering symbol advancing at every interval start
  {
    constexpr uint32_t kWpl = 64 / G;  // 64-bit start words per lane
    uint32_t pc = 0;
#pragma unroll
    for (uint32_t q = 0; q < kWpl; q++) pc += __popcll(sm.u.b.starts[kWpl * g + q]);
    int rank = (int)(grp_incl_sum<G>(pc) - pc) - 1;
    uint32_t cur = (on && rank >= 0) ? sm.u.b.by_rank[rank] : 0u;
    uint32_t* out32 = reinterpret_cast<uint32_t*>(sm.sym) + 16 * kWpl * g;
    if (on) {
#pragma unroll
      for (uint32_t q = 0; q < kWpl; q++) {
        const unsigned long long w = sm.u.b.starts[kWpl * g + q];
        for (uint32_t r = 0; r < 16; r++) {
          uint32_t word = 0;
#pragma unroll
          for (uint32_t b = 0; b < 4; b++) {
            if ((w >> (4 * r + b)) & 1) cur = sm.u.b.by_rank[++rank];
            word |= cur << (8 * b);
          }
          out32[16 * q + r] = word;
        }
      }
    }
  }
  wave_sync();  // the build scratch is dead from here: the ring reuses it
  // ---- states and word ring
  const uint8_t* wsrc = src + tsz + 4 * W;
  const uint32_t nwords = on ? (clen - tsz - 4 * W) >> 1 : 0;
  uint32_t x = (on && g < W) ? ld32(src + tsz + 4 * g) : kL;
  if (on && g < W && x < kL) bad = true;
  bad = grp_any<G>(bad, h);
  on = on && !bad;
  const uintptr_t a0 = (uintptr_t)wsrc & ~(uintptr_t)7;
  const uint32_t hw = (uint32_t)((uintptr_t)wsrc - a0) >> 1;  // word 0 in chunk 0
  const uint32_t nchunks = on ? (2 * (hw + nwords) + 8 * G - 1) / (8 * G) : 0;
  const ACE_GLOBAL u32x2* gch = gp(reinterpret_cast<const u32x2*>(a0));
  uint32_t committed = 0;
  for (; committed < 2 && committed < nchunks; committed++)
    sm.u.ring[(committed & 1) * G + g] = gch[committed * G + g];
  u32x2 pf;
  pf.x = 0;
  pf.y = 0;
  if (committed < nchunks) pf = gch[committed * G + g];
  wave_sync();
  const uint16_t* ring16 = reinterpret_cast<const uint16_t*>(sm.u.ring);
  uint32_t rp = hw;  // ring position (in words) of the next unread word
  const bool lane_on = on && g < W;
  const uint32_t my_steps = on ? (n + W - 1) / W : 0;
  const uint32_t nsteps = uniform(G == 64 ? my_steps : max(my_steps, (uint32_t)__shfl_xor(my_steps, 32, 64)));
  // Each step's decoded symbols go straight to their output bytes: lane j
  // writes byte t*W + j, so a step is one coalesced W-byte store.
  constexpr uint32_t kU = 4;  // steps per ring check in the main loop
  uint8_t* op = dst + g;      // this lane's next output byte
  // Makes room for `steps` more steps in the word ring.
  auto prepare = [&](uint32_t steps) {
    const bool refill = rp + steps * W > committed * kChunkW && committed < nchunks;  // group-uniform
    if (__ballot(refill)) {
      if (refill) {
        sm.u.ring[(committed & 1) * G + g] = pf;
        committed++;
        if (committed < nchunks) pf = gch[committed * G + g];
      }
      wave_sync();
    }
  };
  // One step.  kAll: every lane of the wave holds a state with a symbol in
  // this step, so the renormalisation ballot is the comparison itself.
  auto step = [&](auto all, bool act) {
    constexpr bool kAll = decltype(all)::value;
    const uint32_t slot = x & (kM - 1);
    const uint32_t s = sm.sym[slot];
    const uint32_t e = sm.fc[s];
    const uint32_t xn = __umul24(e >> 16, x >> kProbBits) + (slot - (e & 0xFFFFu));  // low half: cum
    const bool lt = xn < kL;
    const bool need = kAll ? lt : (act && lt);
    const uint64_t m = __builtin_amdgcn_ballot_w64(need);
    const uint32_t mlo = (uint32_t)m, mhi = (uint32_t)(m >> 32);
    const uint32_t pos = __builtin_amdgcn_mbcnt_hi(mhi, __builtin_amdgcn_mbcnt_lo(G == 64 || h == 0 ? mlo : 0u, rp));
    uint32_t wd = ring16[(pos & (2 * kChunkW - 1))];
    ACE_OPAQUE(wd);  // read for every lane: keeps the update branch-free
    const uint32_t xa = (kAll || act) ? xn : x;
    x = need ? ((xn << 16) | wd) : xa;
    rp += (uint32_t)(G == 64 ? __popcll(m) : __popc(h ? mhi : mlo));
    if (kAll || act) st8(op, (uint8_t)s);
    op += kAll ? G : W;  // kAll: W == G
  };
  // main loop: steps where every state of both groups has a symbol, kU at a
  // time with one check; then the ragged tail one step at a time
  const uint32_t my_full = on ? n / W : 0;
  const uint32_t t_full =
      uniform(G == 64 ? my_full : min(my_full, (uint32_t)__shfl_xor(my_full, 32, 64))) & ~(kU - 1);
  uint32_t t = 0;
  if (W == G) {  // every lane holds a state: no per-lane activity in the main loop
    for (; t < t_full; t += kU) {
      prepare(kU);
#pragma unroll
      for (uint32_t u = 0; u < kU; u++) step(std::true_type{}, true);
    }
  } else {
    for (; t < t_full; t += kU) {
      prepare(kU);
#pragma unroll
      for (uint32_t u = 0; u < kU; u++) step(std::false_type{}, lane_on);
    }
  }
  for (; t < nsteps; t++) {
    prepare(1);
    step(std::false_type{}, lane_on && g + t * W < n);
  }
  if (on && (rp - hw != nwords || (g < W && x != kL))) bad = true;
  return grp_any<G>(bad, h);
}

// Kernel (a): grid (ceil(n_plan / (64/G)), 3); each wavefront decodes stream
// t of 64/G consecutive plan entries.  LIT goes to lit + plan_index * B, LEN
// to lens + 4 * seq_base and OFF to offs + ow * seq_base; raw streams are
// left in place (the expansion reads them there).  Also records where each
// block's bytes will live.
template <uint32_t G>
__global__ __launch_bounds__(64) void k_rans(DecodeArgs a, uint32_t plan_lo, uint32_t plan_hi, int lv_lo,
                                             int lv_hi) {
  __shared__ RansGroup<G> sm[64 / G];
  const uint32_t lane = threadIdx.x, h = lane / G, g = lane % G, t = blockIdx.y;
  if (lv_lo >= 0) {  // the plan range of levels [lv_lo, lv_hi), from device memory
    plan_lo = a.lvl_dev[lv_lo];
    plan_hi = a.lvl_dev[lv_hi];
  } else if (a.n_plan_dev) {
    plan_hi = *a.n_plan_dev;
  }
  const uint32_t i = plan_lo + blockIdx.x * (64 / G) + h;
  bool on = i < plan_hi;
  if (!__ballot(on)) return;
  // only the fields this kernel needs (no whole-entry copy: raw[t] is
  // indexed by the grid's y coordinate)
  const PlanEntry* pp = a.plan + (on ? i : 0);
  uint32_t blk = 0, seq_base = 0;
  uint64_t pdst = 0, pay = 0, raw_t = kCoded;
  if (on) {
    blk = pp->block;
    seq_base = pp->seq_base;
    pdst = pp->dst;
    pay = pp->pay;
    raw_t = pp->raw[t];
  }
  if (on && t == 0 && g == 0) a.loc[blk] = a.dst_base + pdst;
  on = on && raw_t == kCoded;
  if (!__ballot(on)) return;  // raw streams are read in place by the expansion
  const uint8_t* d = a.arch + pay + kSDesc * t;
  uint32_t n = 0, clen = 0, off = 0;
  if (on) {
    n = ld32(d + 4);
    clen = ld32(d + 8);
    off = ld32(d + 12);
  }
  uint8_t* dst = t == 0 ? a.lit + (uint64_t)i * a.B
               : t == 1 ? a.lens + 4ull * seq_base
                        : a.offs + (uint64_t)a.ow * seq_base;
  const uint8_t* src = a.arch + pay + off;
  const unsigned long long c0 = a.trace ? (unsigned long long)wall_clock64() : 0ull;
  if (rans_decode_group<G>(src, clen, n, a.W, dst, sm[h], g, h, on) && g == 0) flag(a.err, kErrCorrupt);
  if (a.trace && on && g == 0) {
    a.trace[8ull * i + 2 + 2 * t] = c0;
    a.trace[8ull * i + 3 + 2 * t] = (unsigned long long)wall_clock64();
  }
}

// ---------------------------------------------------------------------------
// Match layer: expansion of one block by a workgroup of kThreads threads.
//
// Sequences are taken 2*kThreads at a time (two per thread, so a 16 KiB
// block is usually one tile).  A workgroup scan of L_k + M_k and L_k gives
// every sequence its block-relative start and its first literal.  Match byte
// i of sequence k reads absolute position O_k + (i mod d_k), d_k = (match
// start) - O_k, so all of a match's bytes come from its source span
// [O_k, O_k + min(M_k, d_k)), which lies before the match.  Each span is
// resolved to one address in memory whenever it can be:
//   * inside one earlier block: that block's location (the block's
//     dependency list is cached in LDS once per block; the location is
//     computed in a whole-archive decode, else read from the location table);
//   * inside an earlier tile of this block: the output itself;
//   * inside this tile: pointer jumping over sequences.  A span inside a
//     literal run resolves to the literal stream; a span inside one period
//     of another match's bytes points at that match's span, and pointers are
//     doubled (a pointer to a pointer becomes one) until each reaches a
//     resolved span, so a chain of n such matches takes log2(n) rounds.
// Output is then produced in 16-byte chunks: a chunk of one literal run or
// of one resolved, non-wrapping match is one 16-byte load (global loads take
// any byte alignment on this target) and one store; the
// others are assembled byte by byte, every byte's address first and then the
// loads together.  Spans that straddle sequences or blocks take the slow
// path: follow the source back until it reaches a literal, a resolved span,
// an earlier tile or an earlier block; each step moves strictly backwards.
// ---------------------------------------------------------------------------
constexpr uint32_t kPoison = 1u, kSlow = 2u, kPend = 4u, kExt = 8u;
constexpr uint32_t kUnres = kPoison | kSlow | kPend;  // flags of a span without an address
constexpr uint32_t kDepCache = 896;  // dependency lists cached in LDS per block (longer: read from HBM)
constexpr uint32_t kMaxJumps = 12;   // pointer-doubling rounds (chains up to 4096)

template <uint32_t kThreads>
struct ExpandSmem {
  static constexpr uint32_t kSeq = 2 * kThreads;    // sequences per tile (two per thread)
  static constexpr uint32_t kRound = 4 * kThreads;  // 16-byte chunks sorted per round
  static constexpr uint32_t kSeqBits = kThreads <= 64 ? 7 : kThreads <= 128 ? 8 : kThreads <= 256 ? 9 : 10;
  uint32_t list[kRound];  // per-byte chunks: chunk << kSeqBits | sequence
  uint32_t cseq[kRound];  // marks: the last sequence starting in each chunk (0 = none)
  uint32_t nbyte;
  uint32_t dst[kSeq];     // block-relative start of the sequence
  uint32_t lm[kSeq];      // L | M << 16
  uint32_t lit[kSeq];     // index of the sequence's first literal in the literal stream
  uint32_t dfl[kSeq];     // min(d, 2^24 - 1) | flags << 24
  uint32_t win[kSeq];     // readable bytes around src0: back (0..31) | forward << 5
  uint32_t ptr[kSeq];     // pending span: span of sequence (ptr >> 16) from offset (ptr & 0xFFFF)
  uint64_t src0[kSeq];    // address of the first byte of a resolved span
  uint32_t deps[kDepCache];
  uint32_t scan[32];
};

// Inclusive scans of four values over the workgroup (kThreads threads):
// v[j] becomes the sum of v[j] over threads 0..tid, t[j] the total.
template <uint32_t kThreads>
__device__ __forceinline__ void wg_scan4(uint32_t (&v)[4], uint32_t (&t)[4], uint32_t* sh) {
  constexpr uint32_t kW = kThreads / 64;
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (uint32_t j = 0; j < 4; j++) v[j] = wave_incl_sum(v[j], lane);
  if (kW == 1) {
#pragma unroll
    for (uint32_t j = 0; j < 4; j++) t[j] = lane63(v[j]);
    return;
  }
  __syncthreads();
  if (lane == 63) {
#pragma unroll
    for (uint32_t j = 0; j < 4; j++) sh[4 * w + j] = v[j];
  }
  __syncthreads();
#pragma unroll
  for (uint32_t j = 0; j < 4; j++) {
    uint32_t o = 0, tot = 0;
    for (uint32_t q = 0; q < kW; q++) {
      const uint32_t x = sh[4 * q + j];
      if (q < w) o += x;
      tot += x;
    }
    v[j] += o;
    t[j] = tot;
  }
}

// Running maximum over kRound = 4 * kThreads values held strided: thread t
// holds the values at positions t + j * kThreads (j < 4).  In place,
// v[j] = max(carry, every value at or before its position); returns the
// maximum of all of them and carry.  One barrier (none for one wavefront);
// the caller must order any earlier reads of sh before it.
template <uint32_t kThreads>
__device__ __forceinline__ uint32_t wg_max_scan_strided4(uint32_t (&v)[4], uint32_t carry, uint32_t* sh) {
  constexpr uint32_t kW = kThreads / 64;
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (uint32_t j = 0; j < 4; j++) v[j] = wave_incl_max(v[j]);
  uint32_t run = carry;
  if (kW == 1) {
#pragma unroll
    for (uint32_t j = 0; j < 4; j++) {
      const uint32_t tot = lane63(v[j]);
      v[j] = max(v[j], run);
      run = max(run, tot);
    }
    return run;
  }
  if (lane == 63) {
#pragma unroll
    for (uint32_t j = 0; j < 4; j++) sh[4 * w + j] = v[j];
  }
  __syncthreads();
#pragma unroll
  for (uint32_t j = 0; j < 4; j++) {
    uint32_t before = run, tot = run;
    for (uint32_t q = 0; q < kW; q++) {
      const uint32_t x = sh[4 * q + j];
      if (q < w) before = max(before, x);
      tot = max(tot, x);
    }
    v[j] = max(v[j], before);
    run = tot;
  }
  return run;
}

__device__ __forceinline__ uint32_t find_seq(const uint32_t* sdst, uint32_t cnt, uint32_t p) {
  uint32_t lo = 0, hi = cnt;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (sdst[mid] <= p) lo = mid; else hi = mid;
  }
  return lo;
}

// Index of c in the ascending list, or -1.
// Branch-free: pos becomes the count of entries below c by binary lifting
// (steps 2^k .. 1, the largest 2^k <= cnt), so the step count depends only
// on cnt, which is uniform over the workgroup.
template <typename P>
__device__ __forceinline__ int dep_index(P deps, uint32_t cnt, uint32_t c) {
  if (cnt == 0) return -1;
  uint32_t pos = 0;
  for (uint32_t step = 1u << (31 - __clz(cnt)); step; step >>= 1)
    if (pos + step <= cnt && deps[pos + step - 1] < c) pos += step;
  return pos < cnt && deps[pos] == c ? (int)pos : -1;
}

struct BlockCtx {
  uint64_t bs;       // absolute start of the block
  uint32_t blen, n_lit, d0, cnt, dep_cnt;
  uint32_t t0, ow;   // the tile's first sequence; offset width in bytes
  uint8_t* out;      // the block's first byte
  const uint8_t* lit;   // the block's literal stream
  const uint8_t* offs;  // the block's offset stream (O_k of sequence k at ow * k)
  bool ext_ok;
};

// Location of the first byte of earlier block blk: computed in a
// whole-archive decode (blocks back to back in the output), else read from
// the location table.
__device__ __forceinline__ uint64_t blk_loc(const DecodeArgs& a, uint64_t blk) {
  return a.loc_linear ? a.dst_base + blk * a.B : *gp(a.loc + blk);
}

// Slow path: the address of the byte at block-relative p, following sources
// back to a literal, a resolved span, an earlier tile of this block or an
// earlier block; null when the byte is to be written as zero (a failed
// format rule, or an earlier block that was never published).  Reads LDS,
// the offset stream and (outside whole-archive decodes) the location table.
template <uint32_t kThreads>
__device__ const uint8_t* resolve_addr(const DecodeArgs& a, const ExpandSmem<kThreads>& sm,
                                       const BlockCtx& c, uint32_t p, uint32_t& n_ext) {
  for (;;) {
    const uint32_t s = find_seq(sm.dst, c.cnt, p);
    const uint32_t fl = sm.dfl[s] >> 24;
    if (fl & kPoison) return nullptr;
    const uint32_t r = p - sm.dst[s];
    const uint32_t Ls = sm.lm[s] & 0xFFFFu;
    if (r < Ls) return c.lit + sm.lit[s] + r;
    const uint32_t ii = r - Ls, d = sm.dfl[s] & 0xFFFFFFu;
    const uint32_t im = ii < d ? ii : ii % d;
    if (!(fl & kUnres)) {
      if (fl & kExt) n_ext++;
      return reinterpret_cast<const uint8_t*>(sm.src0[s] + im);
    }
    const uint32_t k = c.t0 + s;  // O is read back from the token stream (rare path)
    const uint64_t src = (c.ow == 4 ? (uint64_t)ld32(c.offs + 4ull * k) : ld64(c.offs + 8ull * k)) + im;
    if (src < c.bs) {
      if (!c.ext_ok) return nullptr;
      n_ext++;
      const uint64_t blk = blk_of(a, src);
      return reinterpret_cast<const uint8_t*>(blk_loc(a, blk)) + (src - blk * a.B);
    }
    const uint32_t q = (uint32_t)(src - c.bs);
    if (q < c.d0) return c.out + q;
    p = q;
  }
}

// Block-relative position of slow byte u of the tile: slot k's slow bytes
// end at sm.ptr[k] (its match bytes, numbered in sequence order).
template <uint32_t kThreads>
__device__ __forceinline__ uint32_t slow_pos(const ExpandSmem<kThreads>& sm, const BlockCtx& c, uint32_t u) {
  uint32_t lo = 0, hi = c.cnt;  // first slot whose slow-byte end exceeds u
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (sm.ptr[mid] > u) hi = mid; else lo = mid + 1;
  }
  const uint32_t Mk = sm.lm[lo] >> 16, Lk = sm.lm[lo] & 0xFFFFu;
  return sm.dst[lo] + Lk + (u - (sm.ptr[lo] - Mk));
}

// 16 bytes from any byte address (one global load: this target's global
// loads take any alignment).
typedef u32x4 u32x4_a1 __attribute__((aligned(1)));
__device__ __forceinline__ uint4 ld16u(const uint8_t* p) {
  const u32x4 v = *reinterpret_cast<const ACE_GLOBAL u32x4_a1*>(gp(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st16u(uint8_t* p, uint4 v) {  // any byte alignment
  u32x4 w;
  w.x = v.x;
  w.y = v.y;
  w.z = v.z;
  w.w = v.w;
  *reinterpret_cast<ACE_GLOBAL u32x4_a1*>(gp(p)) = w;
}

// Copies len bytes of the decoded data from absolute position lo to dst.
// Each thread takes four 16-byte chunks per step (a blockDim.x * 16 stride
// apart, so every load and store instruction is coalesced), issues the loads
// of those whose 16 source bytes lie in one block, then the stores; chunks
// that cross a block edge or the end go byte by byte.  loc[c] is block c's
// location.
__device__ __forceinline__ void copy_range(const DecodeArgs& a, const uint64_t* loc, uint64_t lo,
                                           uint64_t len, uint8_t* dst) {
  constexpr uint32_t kU = 4;
  const uint64_t stride = (uint64_t)blockDim.x * 16;
  for (uint64_t j0 = threadIdx.x * 16ull; j0 < len; j0 += kU * stride) {
    const uint8_t* src[kU];
    bool fast[kU];
#pragma unroll
    for (uint32_t u = 0; u < kU; u++) {
      const uint64_t j = j0 + u * stride, pos = lo + j;
      const uint64_t c = blk_of(a, pos);
      fast[u] = j + 16 <= len && pos + 16 <= (c + 1) * a.B;
      src[u] = fast[u] ? reinterpret_cast<const uint8_t*>(*gp(loc + c)) + (pos - c * a.B) : nullptr;
    }
    uint4 v[kU];
#pragma unroll
    for (uint32_t u = 0; u < kU; u++) v[u] = fast[u] ? ld16u(src[u]) : make_uint4(0, 0, 0, 0);
#pragma unroll
    for (uint32_t u = 0; u < kU; u++) {
      const uint64_t j = j0 + u * stride;
      if (fast[u]) {
        st16u(dst + j, v[u]);
      } else if (j < len) {
        uint64_t pos = lo + j, c = blk_of(a, pos), cend = (c + 1) * a.B;
        const uint8_t* base = reinterpret_cast<const uint8_t*>(*gp(loc + c)) - c * a.B;
        const uint64_t jn = j + 16 < len ? j + 16 : len;
        for (uint64_t q = j; q < jn; q++, pos++) {
          if (pos >= cend) {
            c++;
            cend += a.B;
            base = reinterpret_cast<const uint8_t*>(*gp(loc + c)) - c * a.B;
          }
          st8(dst + q, ld8(base + pos));
        }
      }
    }
  }
}

// Readable bytes around a resolved span's address: back (capped at 31) and
// forward (capped at 2^26).
__device__ __forceinline__ uint32_t win_pack(uint64_t back, uint64_t fwd) {
  return (uint32_t)(back < 31 ? back : 31) | ((uint32_t)(fwd < (1ull << 26) ? fwd : (1ull << 26)) << 5);
}

// Byte mask (as bit mask of dword j's four bytes) of chunk bytes [lo, hi).
__device__ __forceinline__ uint32_t dword_mask(uint32_t j, uint32_t lo, uint32_t hi) {
  uint32_t m = 0;
#pragma unroll
  for (uint32_t b = 0; b < 4; b++) {
    const uint32_t x = 4 * j + b;
    m |= (x >= lo && x < hi) ? (0xFFu << (8 * b)) : 0u;
  }
  return m;
}

// Segment path for a 16-byte output chunk [cb, cb+16) inside the tile: the
// chunk is cut at literal/match and sequence boundaries into at most four
// segments over at most two sequences.  Each segment's source, shifted so
// that its byte j lines up with output byte j, is one 16-byte load (all
// issued before any is used), merged by byte mask.  Bytes of slow spans are left as placeholders (the
// slow pass writes them), bytes of poisoned sequences as zeros.  Returns
// false (the caller takes the per-byte path) for a period wrap inside a
// segment, a third sequence, or a source window that is not known readable.
template <uint32_t kThreads>
__device__ __forceinline__ bool seg_chunk(const ExpandSmem<kThreads>& sm, const BlockCtx& c, uint32_t cb,
                                          uint32_t s, uint32_t d1, uint32_t (&out)[4]) {
  constexpr uint32_t kC = 4;  // candidate segments: (literal, match) x 2 sequences
  uint64_t V[kC];
  uint32_t lo[kC], hi[kC];
  bool load[kC];
  uint32_t x = cb;
  bool ok = true;
  // the two candidate sequences' fields, read at once (indices clamped into
  // the tile arrays; values past c.cnt are never used)
  constexpr uint32_t kSeq = ExpandSmem<kThreads>::kSeq;
  const uint32_t s1 = s + 1 < kSeq ? s + 1 : s, s2 = s + 2 < kSeq ? s + 2 : s;
  const uint32_t dst_q[3] = {sm.dst[s], sm.dst[s1], sm.dst[s2]};
  const uint32_t lm_q[2] = {sm.lm[s], sm.lm[s1]}, dfl_q[2] = {sm.dfl[s], sm.dfl[s1]};
  const uint32_t lit_q[2] = {sm.lit[s], sm.lit[s1]}, win_q[2] = {sm.win[s], sm.win[s1]};
  const uint64_t src_q[2] = {sm.src0[s], sm.src0[s1]};
#pragma unroll
  for (uint32_t q = 0; q < 2; q++) {
    load[2 * q] = load[2 * q + 1] = false;
    lo[2 * q] = hi[2 * q] = lo[2 * q + 1] = hi[2 * q + 1] = 0;
    V[2 * q] = V[2 * q + 1] = 0;
    const uint32_t sq = s + q;
    if (x < cb + 16 && sq < c.cnt) {
      const uint32_t sd = dst_q[q];
      const uint32_t se = sq + 1 < c.cnt ? dst_q[q + 1] : d1;
      const uint32_t L = lm_q[q] & 0xFFFFu;
      const uint32_t dfl = dfl_q[q], f = dfl >> 24, d = dfl & 0xFFFFFFu;
      const uint32_t end = se < cb + 16 ? se : cb + 16;
      if (f & kPoison) {
        lo[2 * q] = x - cb;  // zeros: a segment with no load
        hi[2 * q] = end - cb;
        x = end;
      } else {
        if (x < sd + L) {  // literal run
          const uint32_t h = sd + L < end ? sd + L : end;
          const uint8_t* A = c.lit + lit_q[q] + (x - sd);
          V[2 * q] = (uint64_t)(uintptr_t)A - (x - cb);
          lo[2 * q] = x - cb;
          hi[2 * q] = h - cb;
          load[2 * q] = true;  // literal streams are readable 31 bytes before and 16 after
          x = h;
        }
        if (x < end) {  // match part
          const uint32_t ii0 = x - (sd + L);
          lo[2 * q + 1] = x - cb;
          hi[2 * q + 1] = end - cb;
          if (!(f & kUnres)) {
            const uint64_t A = src_q[q] + ii0;
            const uint64_t v = A - (x - cb);
            const uint32_t wn = win_q[q], back = (wn & 31u) + ii0, fwd = (wn >> 5) - ii0;
            const uint32_t need_back = x - cb;  // bytes read before the segment's source
            ok = ok && ii0 + (end - x) <= d && need_back <= back && 16 - need_back <= fwd;
            V[2 * q + 1] = v;
            load[2 * q + 1] = true;
          }
          x = end;
        }
      }
    }
  }
  if (!ok || x < cb + 16) return false;
  uint4 wv[kC];
#pragma unroll
  for (uint32_t k = 0; k < kC; k++)
    wv[k] = load[k] ? ld16u(reinterpret_cast<const uint8_t*>(V[k])) : make_uint4(0, 0, 0, 0);
#pragma unroll
  for (uint32_t j = 0; j < 4; j++) out[j] = 0;
#pragma unroll
  for (uint32_t k = 0; k < kC; k++) {
    const uint32_t v4[4] = {wv[k].x, wv[k].y, wv[k].z, wv[k].w};
#pragma unroll
    for (uint32_t j = 0; j < 4; j++) {
      const uint32_t m = dword_mask(j, lo[k], hi[k]);
      out[j] = (out[j] & ~m) | (v4[j] & m);
    }
  }
  return true;
}

// Expands plan entry i with kThreads threads.  Sources in earlier blocks must
// be complete and visible (unless ext_ok is false, after a timed-out wait).
template <uint32_t kThreads>
__device__ __forceinline__ void expand_block(const DecodeArgs& a, uint32_t i, ExpandSmem<kThreads>& sm,
                                             bool ext_ok = true) {
  constexpr uint32_t kSeq = ExpandSmem<kThreads>::kSeq, kRound = ExpandSmem<kThreads>::kRound;
  constexpr uint32_t kSB = ExpandSmem<kThreads>::kSeqBits, kSM = (1u << kSB) - 1;
  static_assert(kSeq <= (1u << kSB), "sequence index must fit its field");
  const uint32_t tid = threadIdx.x;
  const PlanEntry pe = a.plan[i];
  const uint32_t b = pe.block;
  const uint32_t n_seq = pe.n_seq, dep_off = pe.dep_off, dep_cnt = pe.dep_cnt;
  const uint32_t* deps = reinterpret_cast<const uint32_t*>(a.arch + kHdr + (uint64_t)kBlk * a.n_blocks) + dep_off;
  // each stream is read in place when stored raw, else from its decoded copy
  BlockCtx c;
  c.n_lit = pe.n_lit;
  c.bs = (uint64_t)b * a.B;
  c.blen = (uint32_t)((a.n_total - c.bs) < a.B ? (a.n_total - c.bs) : a.B);
  c.out = reinterpret_cast<uint8_t*>(a.dst_base + pe.dst);
  c.ext_ok = ext_ok;
  c.dep_cnt = dep_cnt;
  c.lit = pe.raw[0] != kCoded ? a.arch + pe.raw[0] : a.lit + (uint64_t)i * a.B;
  const uint8_t* lens = pe.raw[1] != kCoded ? a.arch + pe.raw[1] : a.lens + 4ull * pe.seq_base;
  const uint8_t* offs = pe.raw[2] != kCoded ? a.arch + pe.raw[2] : a.offs + (uint64_t)a.ow * pe.seq_base;
  c.offs = offs;
  c.ow = a.ow;
  const bool aligned = (((uintptr_t)c.out) & 15) == 0;
  const bool cached = dep_cnt <= kDepCache;
  uint32_t carry_pos = 0, carry_lit = 0, n_ext = 0;
  bool bad = false;
  // the chunk marks start cleared (each thread clears the entries it later
  // reads, right after reading them), ordered before the first marks by the
  // barriers of the token phase
#pragma unroll
  for (uint32_t j = 0; j < 4; j++) sm.cseq[tid + j * kThreads] = 0;
  if (tid == 0) sm.nbyte = 0;
  for (uint32_t t0 = 0; t0 < n_seq; t0 += kSeq) {
    // ---- two sequences per thread: tokens, scans, first classification
    uint32_t L[2] = {0, 0}, M[2] = {0, 0};
    uint64_t O[2] = {0, 0};
#pragma unroll
    for (uint32_t h = 0; h < 2; h++) {
      const uint32_t k = t0 + tid + h * kThreads;  // slot tid + h * kThreads
      if (k < n_seq) {
        const uint32_t lm = ld32(lens + 4ull * k);
        L[h] = lm & 0xFFFFu;
        M[h] = lm >> 16;
        O[h] = a.ow == 4 ? (uint64_t)ld32(offs + 4ull * k) : ld64(offs + 8ull * k);
      }
    }
    if (t0 == 0) {
      // the block's dependency list, once, in LDS (issued after the first
      // tile's token loads, so the latencies overlap)
      for (uint32_t j = tid; j < (cached ? dep_cnt : 0u); j += kThreads) sm.deps[j] = deps[j];
    }
    // positions in sequence order: slots 0..kThreads-1 first, then the rest
    uint32_t sv[4] = {L[0] + M[0], L[0], L[1] + M[1], L[1]}, st[4];
    wg_scan4<kThreads>(sv, st, sm.scan);
    const uint32_t tp = st[0] + st[2], tl = st[1] + st[3];
    const uint32_t d0 = carry_pos;
    c.d0 = d0;
    c.t0 = t0;
    c.cnt = (n_seq - t0) < kSeq ? (n_seq - t0) : kSeq;
    const uint32_t pos_h[2] = {carry_pos + sv[0] - (L[0] + M[0]), carry_pos + st[0] + sv[2] - (L[1] + M[1])};
    const uint32_t lit_h[2] = {carry_lit + sv[1] - L[0], carry_lit + st[1] + sv[3] - L[1]};
    uint32_t fl_h[2] = {0, 0};
#pragma unroll
    for (uint32_t h = 0; h < 2; h++) {
      const uint32_t k = t0 + tid + h * kThreads, slot = tid + h * kThreads;
      const uint32_t pos = pos_h[h], litk = lit_h[h];
      uint32_t fl = 0, dist = 0, win = 0;
      uint64_t src0 = 0;
      if (k < n_seq) {
        const uint64_t mabs = c.bs + pos + L[h];
        if ((uint64_t)pos + L[h] + M[h] > c.blen || (uint64_t)litk + L[h] > c.n_lit) fl = kPoison;
        if (M[h] && !fl) {
          if (O[h] >= mabs) {
            fl = kPoison;
          } else {
            const uint64_t dd = mabs - O[h];
            dist = (uint32_t)(dd < 0xFFFFFFull ? dd : 0xFFFFFFull);
            const uint64_t span_end = O[h] + (M[h] < dd ? M[h] : dd);  // bytes actually read
            // every earlier block the span touches must be a listed
            // dependency; blocks that lie back to back in memory (always so
            // in a whole-archive decode) make one contiguous source
            bool contiguous = ext_ok;
            uint64_t loc0 = 0;
            if (O[h] < c.bs) {
              const uint64_t end = span_end < c.bs ? span_end : c.bs;
              const uint64_t b0 = blk_of(a, O[h]);
              for (uint64_t blk = b0; blk * a.B < end; blk++) {
                const int di = cached ? dep_index(sm.deps, dep_cnt, (uint32_t)blk)
                                      : dep_index(gp(deps), dep_cnt, (uint32_t)blk);
                if (di < 0) {
                  fl = kPoison;
                  break;
                }
                if (contiguous) {
                  const uint64_t lb = blk_loc(a, blk);
                  if (blk == b0) loc0 = lb;
                  else contiguous = lb == loc0 + (blk - b0) * a.B;
                }
              }
            }
            if (!fl) {
              const uint64_t b0 = blk_of(a, O[h]);
              if (span_end <= c.bs && contiguous) {
                const uint64_t off = O[h] - b0 * a.B;  // earlier blocks, one run of memory
                const uint64_t nblk = blk_of(a, span_end - 1) - b0 + 1;
                src0 = loc0 + off;
                win = win_pack(off, nblk * a.B - off);
                fl = kExt;
                n_ext += M[h];
              } else if (O[h] >= c.bs && span_end - c.bs <= d0) {
                const uint64_t q = O[h] - c.bs;  // an earlier tile of this block
                src0 = (uint64_t)(uintptr_t)c.out + q;
                win = win_pack(q, c.blen - q);
              } else if (O[h] >= c.bs + d0) {
                fl = kPend;  // inside this tile: resolved below
              } else {
                fl = kSlow;
              }
            }
          }
        } else if (!M[h] && O[h] != 0) {
          bad = true;
        }
        if (fl & kPoison) bad = true;
      }
      fl_h[h] = fl;
      sm.dst[slot] = pos;
      sm.lm[slot] = L[h] | (M[h] << 16);
      sm.lit[slot] = litk;
      sm.dfl[slot] = dist | (fl << 24);
      sm.win[slot] = win;
      sm.src0[slot] = src0;
    }
    __syncthreads();
    // ---- spans inside this tile: a literal run resolves at once; a span
    // inside one period of another match points at that match's span
#pragma unroll
    for (uint32_t h = 0; h < 2; h++) {
      if (!(fl_h[h] & kPend)) continue;
      const uint32_t slot = tid + h * kThreads;
      const uint32_t q = (uint32_t)(O[h] - c.bs);
      const uint32_t dist = sm.dfl[slot] & 0xFFFFFFu;
      const uint32_t sl = M[h] < dist ? M[h] : dist;
      const uint32_t j = find_seq(sm.dst, c.cnt, q);
      const uint32_t r = q - sm.dst[j], Lj = sm.lm[j] & 0xFFFFu, Mj = sm.lm[j] >> 16;
      uint32_t fl = kSlow, ptr = 0;
      uint64_t src0 = 0;
      uint32_t win = 0;
      const bool j_ok = !((sm.dfl[j] >> 24) & kPoison);  // a poisoned run is written as zeros
      if (j_ok && r + sl <= Lj) {
        const uint32_t lp = sm.lit[j] + r;
        src0 = (uint64_t)(uintptr_t)(c.lit + lp);
        win = win_pack(lp, (uint64_t)(c.n_lit - lp) + 4);  // literal streams have readable slack
        fl = 0;
      } else if (j_ok && r >= Lj) {
        const uint32_t off = r - Lj, dj = sm.dfl[j] & 0xFFFFFFu;
        if (off + sl <= Mj && (Mj <= dj || off / dj == (off + sl - 1) / dj)) {
          ptr = (j << 16) | (Mj <= dj ? off : off % dj);
          fl = kPend;
        }
      }
      sm.dfl[slot] = dist | (fl << 24);
      sm.ptr[slot] = ptr;
      sm.src0[slot] = src0;
      sm.win[slot] = win;
      fl_h[h] = fl;
    }
    // ---- pointer doubling
    for (uint32_t round = 0;; round++) {
      const bool pend = (fl_h[0] | fl_h[1]) & kPend;
      if (!__syncthreads_or(pend)) break;
      uint32_t nfl[2] = {fl_h[0], fl_h[1]}, nptr[2] = {0, 0}, nwin[2] = {0, 0};
      uint64_t nsrc[2] = {0, 0};
#pragma unroll
      for (uint32_t h = 0; h < 2; h++) {
        if (!(fl_h[h] & kPend)) continue;
        const uint32_t pt = sm.ptr[tid + h * kThreads], j = pt >> 16, off = pt & 0xFFFFu;
        const uint32_t fj = sm.dfl[j] >> 24;
        if (!(fj & kUnres)) {
          const uint32_t wj = sm.win[j];
          nsrc[h] = sm.src0[j] + off;
          nwin[h] = win_pack((wj & 31u) + off, (wj >> 5) - off);
          nfl[h] = fj & kExt;
          if (fj & kExt) n_ext += M[h];
        } else if ((fj & kPend) && round + 1 < kMaxJumps) {
          const uint32_t pj = sm.ptr[j];
          nptr[h] = (pj & 0xFFFF0000u) | ((pj & 0xFFFFu) + off);
        } else {
          nfl[h] = kSlow;
        }
      }
      __syncthreads();
#pragma unroll
      for (uint32_t h = 0; h < 2; h++) {
        if (!(fl_h[h] & kPend)) continue;
        const uint32_t slot = tid + h * kThreads;
        const uint32_t dist = sm.dfl[slot] & 0xFFFFFFu;
        sm.dfl[slot] = dist | (nfl[h] << 24);
        if (nfl[h] & kPend) {
          sm.ptr[slot] = nptr[h];
        } else if (!(nfl[h] & kUnres)) {
          sm.src0[slot] = nsrc[h];
          sm.win[slot] = nwin[h];
        }
        fl_h[h] = nfl[h];
      }
    }
    // slow sequences' match bytes, numbered: slot k's end in sm.ptr (the
    // pointers are no longer needed)
    uint32_t n_slow = 0;
    {
      uint32_t cv[4] = {(fl_h[0] & kSlow) ? M[0] : 0u, 0u, (fl_h[1] & kSlow) ? M[1] : 0u, 0u}, ct[4];
      wg_scan4<kThreads>(cv, ct, sm.scan);
      sm.ptr[tid] = cv[0];
      sm.ptr[tid + kThreads] = ct[0] + cv[2];
      n_slow = ct[0] + ct[2];
      __syncthreads();
    }
    const uint64_t d1w = (uint64_t)carry_pos + tp;
    const uint32_t d1 = d1w < c.blen ? (uint32_t)d1w : c.blen;
    // ---- output in 16-byte chunks, four per thread per round: copy chunks
    // (one literal run, or one resolved match with no period wrap) are
    // copied where they are
    // classified; per-byte chunks are gathered in a list and spread over
    // the threads, so a wavefront does not pay for both kinds of work
    const uint32_t base = d0 & ~15u;
    const uint32_t nch = d1 > base ? (d1 - base + 15) / 16 : 0;
    uint32_t carry = 0;  // the last sequence marked in earlier rounds
    for (uint32_t k0 = 0; k0 < nch; k0 += kRound) {
      const uint32_t kn = nch - k0 < kRound ? nch - k0 : kRound;
      // the sequence holding each chunk's first byte: every sequence marks
      // the first chunk whose first byte is at or after its start, then a
      // running maximum over the chunks fills the rest.  Thread t reads
      // (and clears) the marks of chunks t + j * kThreads, the chunks it
      // classifies, so the scan leaves each thread exactly its own values.
#pragma unroll
      for (uint32_t h = 0; h < 2; h++) {
        const uint32_t slot = tid + h * kThreads;
        if (slot < c.cnt) {
          const uint32_t ds = sm.dst[slot];
          const uint32_t cm = ds <= d0 ? 0u : (ds - base + 15) / 16;
          if (cm >= k0 && cm < k0 + kn) atomicMax(&sm.cseq[cm - k0], slot);
        }
      }
      __syncthreads();
      uint32_t sqv[4];
#pragma unroll
      for (uint32_t j = 0; j < 4; j++) {
        sqv[j] = sm.cseq[tid + j * kThreads];
        sm.cseq[tid + j * kThreads] = 0;
      }
      // every thread read the previous round's count before the barrier
      // above; this round's additions come after the scan's barrier
      if (tid == 0) sm.nbyte = 0;
      carry = wg_max_scan_strided4<kThreads>(sqv, carry, sm.scan);
      // Phase A (LDS only): classify this thread's four chunks (a copy chunk
      // records its source; the others are appended to a list, one LDS
      // atomic per wavefront) and, in the tile's last round, follow this
      // thread's slow byte back to its source (a slow byte's source is never
      // in this tile's output, so it can be read before the tile is done).
      const bool fold = k0 + kRound >= nch;  // last round: slow bytes written here
      // a copy chunk's 16 source bytes are loaded as soon as it is classified
      // (one load at any byte alignment; other chunks read 16 bytes at c.lit,
      // which is always readable), so the loads are in flight during the
      // rest of the classification, the list barrier and the segment path
      uint4 w[4];
      uint32_t cbv[4];
#pragma unroll
      for (uint32_t j = 0; j < 4; j++) {
        const uint32_t k = k0 + tid + j * kThreads;
        const bool here = k < k0 + kn;
        const uint32_t cb = base + 16 * k;
        // branch-free: every LDS field the decision needs is read at once
        // (sq is a valid slot even for chunks past the tile's end)
        const uint32_t sq = sqv[j] < c.cnt ? sqv[j] : c.cnt - 1;
        const uint32_t dfl = sm.dfl[sq], sd = sm.dst[sq], lmv = sm.lm[sq], litv = sm.lit[sq];
        const uint32_t sn = sm.dst[sq + 1 < kSeq ? sq + 1 : sq];
        const uint64_t s0 = sm.src0[sq];
        const uint32_t fl = dfl >> 24, Ls = lmv & 0xFFFFu;
        const uint32_t end_s = sq + 1 < c.cnt ? sn : d1;
        const uint32_t r0 = cb - sd, ii0 = r0 - Ls;  // used only when the chunk is whole
        const bool whole = here && aligned && cb >= d0 && cb + 16 <= d1 && cb + 16 <= end_s && !(fl & kPoison);
        // all literals (stream data has readable slack), or a resolved match
        // with no period wrap inside the chunk (its 16 source bytes lie in
        // the resolved span, which is readable)
        const bool lit_ok = r0 + 16 <= Ls;
        const bool mat_ok = r0 >= Ls && !(fl & kUnres) && ii0 + 16 <= (dfl & 0xFFFFFFu);
        const bool vec = whole && (lit_ok || mat_ok);
        const uint8_t* src = lit_ok ? c.lit + litv + r0 : reinterpret_cast<const uint8_t*>(s0 + ii0);
        cbv[j] = vec ? cb : 0xFFFFFFFFu;
        w[j] = ld16u(vec ? src : c.lit);  // c.lit is always readable
        const bool byte = here && !vec;
        const uint64_t mb = __builtin_amdgcn_ballot_w64(byte);
        const uint32_t lane = tid & 63;
        const uint32_t leader_b = mb ? (uint32_t)__builtin_ctzll(mb) : 64u;
        uint32_t bb = 0;
        if (lane == leader_b) bb = atomicAdd(&sm.nbyte, (uint32_t)__popcll(mb));
        bb = (uint32_t)__builtin_amdgcn_readlane((int)bb, (int)(leader_b & 63));
        const uint32_t below_b = __builtin_amdgcn_mbcnt_hi((uint32_t)(mb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mb, 0u));
        if (byte) sm.list[bb + below_b] = (k << kSB) | sq;
      }
      uint32_t slow_p = 0xFFFFFFFFu;
      const uint8_t* slow_a = nullptr;
      if (fold && tid < n_slow) {
        slow_p = slow_pos<kThreads>(sm, c, tid);
        slow_a = resolve_addr<kThreads>(a, sm, c, slow_p, n_ext);
      }
      const uint32_t slow_v = slow_a ? (uint32_t)ld8(slow_a) : 0u;
      __syncthreads();
      const uint32_t nby = sm.nbyte;
      // Phase B: the segment path's loads for this thread's first listed
      // chunk, then the stores.
      bool seg_done = false;
      uint32_t seg_cb = 0, o4[4] = {0, 0, 0, 0};
      if (tid < nby) {
        const uint32_t e = sm.list[tid], k = e >> kSB;
        seg_cb = base + 16 * k;
        const uint32_t p0 = seg_cb < d0 ? d0 : seg_cb;
        const uint32_t pe1 = seg_cb + 16 < d1 ? seg_cb + 16 : d1;
        if (aligned && p0 == seg_cb && pe1 == seg_cb + 16)
          seg_done = seg_chunk<kThreads>(sm, c, seg_cb, e & kSM, d1, o4);
      }
#pragma unroll
      for (uint32_t j = 0; j < 4; j++)
        if (cbv[j] != 0xFFFFFFFFu) st16(c.out + cbv[j], w[j]);
      if (seg_done) st16(c.out + seg_cb, make_uint4(o4[0], o4[1], o4[2], o4[3]));
      // per-byte path: listed chunks the segment path declined or that lie
      // beyond the first kThreads entries.  Every byte's source address
      // first, then the 16 loads back to back.  The current sequence's
      // fields stay in registers (LDS is read only when the walk enters the
      // next sequence), and match bytes step their source offset by one,
      // wrapping at the period.  Bytes of slow sequences get a placeholder
      // here; the slow bytes are written after the barrier below.
      for (uint32_t ei = tid; ei < nby; ei += kThreads) {
        if (ei == tid && seg_done) continue;
        const uint32_t e = sm.list[ei], k = e >> kSB;
        const uint32_t cb = base + 16 * k;
        const uint32_t p0 = cb < d0 ? d0 : cb;
        const uint32_t pe1 = cb + 16 < d1 ? cb + 16 : d1;
        uint32_t s = e & kSM;
        if (ei != tid && aligned && p0 == cb && pe1 == cb + 16) {
          uint32_t q4[4];
          if (seg_chunk<kThreads>(sm, c, cb, s, d1, q4)) {
            st16(c.out + cb, make_uint4(q4[0], q4[1], q4[2], q4[3]));
            continue;
          }
        }
        uint32_t sd = 0, se = 0, sL = 0, sf = 0, sdist = 1, im = 0;
        const uint8_t* litp = c.lit;
        uint64_t src0 = 0;
        bool started = false;
        auto view = [&]() {
          sd = sm.dst[s];
          se = s + 1 < c.cnt ? sm.dst[s + 1] : d1;
          sL = sm.lm[s] & 0xFFFFu;
          sf = sm.dfl[s] >> 24;
          sdist = sm.dfl[s] & 0xFFFFFFu;
          litp = c.lit + sm.lit[s];
          src0 = sm.src0[s];
          started = false;
        };
        view();
        // two halves of eight bytes (this path is rare; halves keep its
        // registers below those of the main path)
        uint32_t acc[4] = {0, 0, 0, 0};
#pragma unroll 1
        for (uint32_t hf = 0; hf < 2; hf++) {
          const uint8_t* ad[8];
          uint32_t zero = 0;
#pragma unroll
          for (uint32_t j = 0; j < 8; j++) {
            const uint32_t p = cb + 8 * hf + j;
            const uint8_t* q = nullptr;
            if (p >= p0 && p < pe1) {
              while (p >= se) {
                s++;
                view();
              }
              const uint32_t r = p - sd;
              if (sf & kPoison) {
                q = nullptr;  // a format rule failed: write zeros, read nothing
              } else if (r < sL) {
                q = litp + r;
              } else if (!(sf & kUnres)) {
                if (!started) {
                  const uint32_t ii = r - sL;
                  im = ii < sdist ? ii : ii % sdist;
                  started = true;
                } else if (++im == sdist) {
                  im = 0;
                }
                q = reinterpret_cast<const uint8_t*>(src0 + im);
              }
            }
            zero |= (q == nullptr ? 1u : 0u) << j;
            ad[j] = q == nullptr ? c.lit : q;  // c.lit is always readable
          }
          uint32_t lo4 = 0, hi4 = 0;
#pragma unroll
          for (uint32_t j = 0; j < 8; j++) {
            const uint32_t v = (zero >> j) & 1u ? 0u : (uint32_t)ld8(ad[j]);
            if (j < 4) lo4 |= v << (8 * j);
            else hi4 |= v << (8 * (j - 4));
          }
          acc[2 * hf] = lo4;
          acc[2 * hf + 1] = hi4;
        }
        if (aligned && p0 == cb && pe1 == cb + 16) {
          st16(c.out + cb, make_uint4(acc[0], acc[1], acc[2], acc[3]));
        } else {
#pragma unroll
          for (uint32_t j = 0; j < 16; j++)
            if (cb + j >= p0 && cb + j < pe1) st8(c.out + cb + j, (uint8_t)(acc[j >> 2] >> (8 * (j & 3))));
        }
      }
      // the slow bytes loaded above, after every chunk store of the tile
      // (only its last round resolves them).  The list and the marks are
      // next written after the next round's first barrier.
      if (fold) {
        __syncthreads();
        if (slow_p != 0xFFFFFFFFu) st8(c.out + slow_p, (uint8_t)slow_v);
      }
    }
    // ---- slow pass: the match bytes of slow sequences (spans that straddle
    // sequences, tiles or non-adjacent blocks), one byte per thread, each
    // followed back to its origin
    const uint32_t slow_from = nch > 0 ? kThreads : 0u;  // the first ones went with the last round
    if (n_slow > slow_from) {
      __syncthreads();  // after every chunk store (placeholders included)
      for (uint32_t u = slow_from + tid; u < n_slow; u += kThreads) {
        const uint32_t p = slow_pos<kThreads>(sm, c, u);
        const uint8_t* q = resolve_addr<kThreads>(a, sm, c, p, n_ext);
        st8(c.out + p, q ? ld8(q) : (uint8_t)0);
      }
      __syncthreads();
    }
    carry_pos = (uint32_t)(d1w > 0xFFFFFFFFull ? 0xFFFFFFFFu : d1w);
    carry_lit += tl;
    if ((uint64_t)carry_pos > c.blen) {
      bad = true;
      break;
    }
  }
  if (tid == 0 && (carry_pos != c.blen || carry_lit > c.n_lit)) bad = true;
  if (bad) flag(a.err, kErrCorrupt);
  // one counter update per block, spread over 16 counters
  n_ext = wave_total(n_ext);
  __syncthreads();
  if ((tid & 63) == 0) sm.scan[tid >> 6] = n_ext;
  __syncthreads();
  if (tid == 0) {
    uint32_t sum = 0;
    for (uint32_t w = 0; w < kThreads / 64; w++) sum += sm.scan[w];
    if (sum) atomicAdd(a.ext_bytes + (b & 15), (unsigned long long)sum);
  }
}

template <uint32_t kThreads>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_expand(DecodeArgs a, uint32_t plan_lo, int level) {
  __shared__ ExpandSmem<kThreads> sm;
  uint32_t i = plan_lo + blockIdx.x;
  if (level >= 0) {
    i = a.lvl_dev[level] + blockIdx.x;
    if (i >= a.lvl_dev[level + 1]) return;
  }
  const unsigned long long c0 = a.trace ? (unsigned long long)wall_clock64() : 0ull;
  expand_block<kThreads>(a, i, sm);
  if (a.trace && threadIdx.x == 0) {
    a.trace[8ull * i] = c0;
    a.trace[8ull * i + 1] = (unsigned long long)wall_clock64();
  }
}

// ---------------------------------------------------------------------------
// Kernel (c): one persistent launch decodes a whole plan, level by level,
// driven by counters in device memory: for each dependency level, how many
// of its blocks have been claimed for expansion and how many are finished;
// one counter of entropy decodes claimed (in plan order, so lower levels
// first) and one completion flag per plan entry.
//
// A workgroup expands blocks of the lowest level it has not yet seen
// finish, and moves on to the next level once that level's finished count
// reaches its size.  A block's dependencies all sit at lower levels, so
// every block it expands finds the blocks it copies from complete.  When no
// block of its level is left to claim, it entropy-decodes the next plan
// entry instead, so the entropy layer of later levels runs under the
// expansion of earlier ones (and an expansion whose streams are not decoded
// yet decodes queued entries until they are).  Work is only ever claimed by
// running workgroups and nothing claimed waits on anything claimed later, so
// the launch needs no co-residency and no workgroup count.
//
// Cross-workgroup visibility: a finished item is published by every wave
// issuing an agent-scope release fence (its own stores done, this XCD's L2
// written back), then a barrier, then one atomic increment or store; the
// consumer polls counters and flags with agent-scope atomic loads and issues
// an agent-scope acquire fence in every wave before it reads the published
// bytes.
//
// Every wait is bounded by a count of consecutive idle polls (not by a
// clock).  An expired wait flags kErrTimeout and the workgroup stops waiting
// from then on, as does every workgroup that sees that flag: levels are
// skipped when not finished and expansions no longer read earlier blocks,
// so the launch always drains (its output is then not valid, and ace_check
// reports the timeout).
// ---------------------------------------------------------------------------
constexpr uint32_t kPersistThreads = 128;

union PersistSmem {
  ExpandSmem<kPersistThreads> e;
  RansGroup<64> r[kPersistThreads / 64];
};

// A counter or flag shared across workgroups, read at agent scope.
__device__ __forceinline__ uint32_t coherent_u32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Every wave of the workgroup: its earlier stores complete and visible at
// agent scope; then all waves meet.
__device__ __forceinline__ void publish_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
}
__device__ __forceinline__ void acquire_all() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// Entropy decode of plan entry i's rANS-coded streams (raw streams are read
// in place by the expansion): wave 0 decodes LIT, wave 1 LEN then OFF.  Also
// records where the block's bytes will live.
__device__ void persist_entropy(const DecodeArgs& a, uint32_t i, PersistSmem& sm) {
  const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const PlanEntry* pp = a.plan + i;
  const uint32_t blk = pp->block, seq_base = pp->seq_base;
  const uint64_t pdst = pp->dst, pay = pp->pay;
  if (threadIdx.x == 0) a.loc[blk] = a.dst_base + pdst;
  const uint32_t t_lo = w == 0 ? 0u : 1u, t_hi = w == 0 ? 1u : 3u;
  for (uint32_t t = t_lo; t < t_hi; t++) {
    if (pp->raw[t] != kCoded) continue;  // wave-uniform
    const uint8_t* d = a.arch + pay + kSDesc * t;
    const uint32_t n = ld32(d + 4), clen = ld32(d + 8), off = ld32(d + 12);
    uint8_t* dst = t == 0 ? a.lit + (uint64_t)i * a.B
                 : t == 1 ? a.lens + 4ull * seq_base
                          : a.offs + (uint64_t)a.ow * seq_base;
    const unsigned long long c0 = a.trace ? (unsigned long long)wall_clock64() : 0ull;
    if (rans_decode_group<64>(a.arch + pay + off, clen, n, a.W, dst, sm.r[w], lane, 0, true) && lane == 0)
      flag(a.err, kErrCorrupt);
    if (a.trace && lane == 0) {
      a.trace[8ull * i + 2 + 2 * t] = c0;
      a.trace[8ull * i + 3 + 2 * t] = (unsigned long long)wall_clock64();
    }
  }
}

__global__ __launch_bounds__(kPersistThreads) void k_persist(DecodeArgs a) {
  __shared__ PersistSmem sm;
  __shared__ uint32_t sh_kind, sh_item, sh_give_up;
  enum : uint32_t { kExit, kExpand, kEntropy, kNextLevel, kIdle };
  const uint32_t tid = threadIdx.x;
  const uint32_t n_plan = a.n_plan_dev ? *a.n_plan_dev : a.n_plan;
  uint32_t lvl = 0, idle = 0;  // thread 0's view
  bool give_up = false;
  if (tid == 0) sh_give_up = 0;
  // thread 0 decides the next step for the whole workgroup; entropy items
  // are taken from the shared queue in plan order
  auto take_entropy = [&](uint32_t& k) -> bool {
    if (__hip_atomic_load(a.queue, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= n_plan) return false;
    k = atomicAdd(a.queue, 1u);
    return k < n_plan;
  };
  auto idle_poll = [&]() {
    // back off while idle (the counters polled are shared by every workgroup)
    if (idle < 16) __builtin_amdgcn_s_sleep(2);
    else __builtin_amdgcn_s_sleep(16);
    if (++idle > a.max_polls || (coherent_u32(a.err) & kErrTimeout)) {
      if (!give_up) flag(a.err, kErrTimeout);
      give_up = true;
    }
  };
  auto run_entropy = [&](uint32_t k) {
    persist_entropy(a, k, sm);
    publish_barrier();
    if (tid == 0) __hip_atomic_store(a.done + k, a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  for (;;) {
    if (tid == 0) {
      uint32_t kind = kIdle, item = 0;
      if (lvl >= a.n_lvl) {
        kind = kExit;
      } else {
        const uint32_t lo = a.lvl_dev[lvl], hi = a.lvl_dev[lvl + 1], size = hi - lo;
        if (__hip_atomic_load(a.lvl_claim + lvl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < size) {
          const uint32_t j = atomicAdd(a.lvl_claim + lvl, 1u);
          if (j < size) {
            kind = kExpand;
            item = lo + j;
          }
        }
        if (kind == kIdle) {
          if (give_up || coherent_u32(a.lvl_done + lvl) >= size) kind = kNextLevel;
          else if (take_entropy(item)) kind = kEntropy;
        }
      }
      if (kind == kIdle) idle_poll();
      else idle = 0;
      sh_kind = kind;
      sh_item = item;
      sh_give_up = give_up ? 1u : 0u;
    }
    __syncthreads();
    const uint32_t kind = sh_kind, item = sh_item;
    const bool stop_waiting = sh_give_up != 0;
    __syncthreads();
    if (kind == kExit) break;
    if (kind == kNextLevel) {
      acquire_all();
      if (tid == 0) lvl++;
      continue;
    }
    if (kind == kEntropy) {
      run_entropy(item);
      continue;
    }
    if (kind != kExpand) continue;
    // the entry's streams must be decoded: decode queued entries (plan order
    // reaches this one) until its flag is set
    for (;;) {
      if (tid == 0) {
        uint32_t st = kIdle, k = 0;
        if (give_up || coherent_u32(a.done + item) == a.epoch) st = kExpand;
        else if (take_entropy(k)) st = kEntropy;
        if (st == kIdle) idle_poll();
        else idle = 0;
        sh_kind = st;
        sh_item = k;
        sh_give_up = give_up ? 1u : 0u;
      }
      __syncthreads();
      const uint32_t st = sh_kind, k = sh_item;
      __syncthreads();
      if (st == kExpand) break;
      if (st == kEntropy) run_entropy(k);
    }
    acquire_all();
    const unsigned long long c0 = a.trace ? (unsigned long long)wall_clock64() : 0ull;
    expand_block<kPersistThreads>(a, item, sm.e, !(stop_waiting || sh_give_up));
    if (a.trace && tid == 0) {
      a.trace[8ull * item] = c0;
      a.trace[8ull * item + 1] = (unsigned long long)wall_clock64();
    }
    publish_barrier();
    if (tid == 0) atomicAdd(a.lvl_done + lvl, 1u);
  }
}

// ---------------------------------------------------------------------------
// Copy of decoded ranges (seek clipping and batched gathers): one workgroup
// per item, 16 contiguous bytes per thread per pass, source blocks found via
// the location table.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_copy(DecodeArgs a, const CopyItem* items) {
  const CopyItem it = items[blockIdx.x];
  copy_range(a, a.loc, it.src_abs, it.len, reinterpret_cast<uint8_t*>(it.dst));
}

// ---------------------------------------------------------------------------
// Device-side planning of a seek batch.  Mark the target blocks of every
// request; close the set under the dependency lists level by level from the
// top (dependencies always sit at lower levels); compact the marked blocks,
// in level order, into a plan whose entries decode into workspace slots;
// after the decode, gather each request's range to its output offset.
// Kept blocks (decoded once, in the first pin_base slots) are never marked:
// their locations stay valid, and closures stop at them.
// ---------------------------------------------------------------------------
__global__ void k_bmark(BatchArgs b) {
  const uint64_t n = b.desc[0];
  for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < n;
       r += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t lo = b.desc[2 + 3 * r], hi = b.desc[3 + 3 * r];
    if (hi <= lo || hi > b.n_total) continue;
    for (uint64_t blk = lo / b.B; blk <= (hi - 1) / b.B; blk++)
      if (!b.pin[blk]) b.need[blk] = 1;
  }
}

__global__ void k_bclose(BatchArgs b, uint32_t level) {
  const uint32_t j0 = b.lstart[level], j1 = b.lstart[level + 1];
  for (uint32_t j = j0 + blockIdx.x * blockDim.x + threadIdx.x; j < j1; j += gridDim.x * blockDim.x) {
    const uint32_t blk = b.order[j];
    if (!b.need[blk]) continue;
    const uint8_t* be = b.arch + kHdr + (uint64_t)kBlk * blk;
    const uint32_t dep_off = ld32(be + 20), dep_cnt = ld32(be + 24);
    const uint32_t* deps = reinterpret_cast<const uint32_t*>(b.arch + kHdr + (uint64_t)kBlk * b.n_blocks) + dep_off;
    for (uint32_t k = 0; k < dep_cnt; k++) {
      const uint32_t d = deps[k];
      if (!b.pin[d]) b.need[d] = 1;
    }
  }
}

// One workgroup of 1024 threads: running scans of "needed" and of n_seq.
__global__ __launch_bounds__(1024) void k_bcompact(BatchArgs b) {
  __shared__ uint32_t sh_cnt[16], sh_seq[16];
  __shared__ uint32_t base_cnt, base_seq;
  const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) {
    base_cnt = 0;
    base_seq = 0;
  }
  __syncthreads();
  for (uint32_t j0 = 0; j0 < b.n_blocks; j0 += 1024) {
    const uint32_t j = j0 + tid;
    uint32_t blk = 0, f = 0, ns = 0;
    if (j < b.n_blocks) {
      blk = b.order[j];
      f = b.need[blk] ? 1u : 0u;
      ns = f ? ld32(b.arch + kHdr + (uint64_t)kBlk * blk + 12) : 0u;
    }
    const uint32_t ic = wave_incl_sum(f, lane), is = wave_incl_sum(ns, lane);
    if (lane == 63) {
      sh_cnt[w] = ic;
      sh_seq[w] = is;
    }
    __syncthreads();
    uint32_t oc = base_cnt, os = base_seq, tc = 0, ts = 0;
    for (uint32_t k = 0; k < 16; k++) {
      if (k < w) {
        oc += sh_cnt[k];
        os += sh_seq[k];
      }
      tc += sh_cnt[k];
      ts += sh_seq[k];
    }
    const uint32_t pos = oc + ic - f, seq = os + is - ns;
    if (j < b.n_blocks) b.pre[j] = pos;
    if (f) {
      const uint8_t* be = b.arch + kHdr + (uint64_t)kBlk * blk;
      PlanEntry e{};
      e.block = blk;
      e.seq_base = seq;
      e.dst = (uint64_t)(*b.pin_base + pos) * b.B;
      e.pay = ld64(be);
      e.n_seq = ns;
      e.dep_off = ld32(be + 20);
      e.dep_cnt = ld32(be + 24);
      const uint8_t* d = b.arch + e.pay;
      e.n_lit = ld32(d + 4);
      for (uint32_t t = 0; t < 3; t++)
        e.raw[t] = d[kSDesc * t] == 0 ? e.pay + ld32(d + kSDesc * t + 12) : kCoded;
      b.plan[pos] = e;
    }
    __syncthreads();
    if (tid == 0) {
      base_cnt += tc;
      base_seq += ts;
    }
    __syncthreads();
  }
  for (uint32_t l = tid; l <= b.depth; l += 1024) b.lvl_dev[l] = l < b.depth ? b.pre[b.lstart[l]] : base_cnt;
  if (tid == 0) *b.n_plan_dev = base_cnt;
}

// One workgroup per request: copy [lo, hi) from the decoded slots.
__global__ __launch_bounds__(256) void k_bgather(BatchArgs b, DecodeArgs a) {
  const uint64_t n = b.desc[0];
  const uint64_t r = blockIdx.x;
  if (r >= n) return;
  const uint64_t lo = b.desc[2 + 3 * r], hi = b.desc[3 + 3 * r];
  if (hi <= lo || hi > b.n_total) return;
  uint8_t* dst = reinterpret_cast<uint8_t*>(b.desc[1] + b.desc[4 + 3 * r]);
  copy_range(a, b.loc, lo, hi - lo, dst);
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint64_t n) {
  for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < n;
       j += (uint64_t)gridDim.x * blockDim.x)
    p[j] = v;
}

}  // namespace

// Entropy launch over plan entries [lo, hi), or (lv_lo >= 0) over the plan
// range of levels [lv_lo, lv_hi) read from device memory, with hi - lo
// entries of capacity.
static hipError_t launch_rans_any(const DecodeArgs& a, uint32_t lo, uint32_t hi, int lv_lo, int lv_hi,
                                  uint32_t per_wave, hipStream_t s) {
  if (hi <= lo) return hipSuccess;
  const uint32_t n = hi - lo;
  if (per_wave == 0) per_wave = a.W <= 32 ? 2 : 1;
  if (per_wave == 2 && a.W <= 32)
    hipLaunchKernelGGL(k_rans<32>, dim3((n + 1) / 2, 3), dim3(64), 0, s, a, lo, hi, lv_lo, lv_hi);
  else
    hipLaunchKernelGGL(k_rans<64>, dim3(n, 3), dim3(64), 0, s, a, lo, hi, lv_lo, lv_hi);
  return hipGetLastError();
}

hipError_t launch_rans(const DecodeArgs& a, uint32_t lo, uint32_t hi, uint32_t per_wave, hipStream_t s) {
  return launch_rans_any(a, lo, hi, -1, -1, per_wave, s);
}

// Four-wavefront expansion workgroups the current device holds at once
// (0 if the query fails), cached per device.
static uint32_t expand4_resident() {
  static std::atomic<uint32_t> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  uint32_t v = cache[dev].load(std::memory_order_relaxed);
  if (v) return v;
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_expand<256>, 256, 0) != hipSuccess ||
      cus <= 0 || per_cu <= 0)
    return 0;
  v = (uint32_t)cus * (uint32_t)per_cu;
  cache[dev].store(v, std::memory_order_relaxed);
  return v;
}

hipError_t prepare_expand_shapes() { return expand4_resident() ? hipSuccess : hipErrorUnknown; }

// One expansion launch: grid blocks from plan_lo, or (level >= 0) the plan
// range of that level read from device memory; waves = wavefronts per block,
// 0 = chosen by the launch's size.  While the launch's blocks all fit on the
// device at once as four-wavefront workgroups, one block's latency sets the
// launch's time and four wavefronts per block shorten it; beyond that the
// blocks in flight set it, and two-wavefront workgroups (same registers per
// wavefront, half the LDS per block) keep twice as many.
static hipError_t launch_expand(const DecodeArgs& a, uint32_t grid, uint32_t plan_lo, int level,
                                uint32_t waves, hipStream_t s) {
  if (grid == 0) return hipSuccess;
  if (waves == 0) waves = grid <= expand4_resident() ? 4u : 2u;
  switch (waves) {
    case 1: hipLaunchKernelGGL(k_expand<64>, dim3(grid), dim3(64), 0, s, a, plan_lo, level); break;
    case 4: hipLaunchKernelGGL(k_expand<256>, dim3(grid), dim3(256), 0, s, a, plan_lo, level); break;
    case 8: hipLaunchKernelGGL(k_expand<512>, dim3(grid), dim3(512), 0, s, a, plan_lo, level); break;
    default: hipLaunchKernelGGL(k_expand<128>, dim3(grid), dim3(128), 0, s, a, plan_lo, level); break;
  }
  return hipGetLastError();
}

hipError_t launch_expand_level(const DecodeArgs& a, uint32_t lo, uint32_t hi, uint32_t waves,
                               hipStream_t s) {
  if (hi <= lo) return hipSuccess;
  return launch_expand(a, hi - lo, lo, -1, waves, s);
}

// cap: the largest plan length the launch must cover (the length itself is
// read from device memory)
hipError_t launch_rans_dev(const DecodeArgs& a, uint32_t cap, uint32_t per_wave, hipStream_t s) {
  return launch_rans_any(a, 0, cap, -1, -1, per_wave, s);
}

hipError_t launch_rans_levels_dev(const DecodeArgs& a, uint32_t lv_lo, uint32_t lv_hi, uint32_t width,
                                  uint32_t per_wave, hipStream_t s) {
  return launch_rans_any(a, 0, width, (int)lv_lo, (int)lv_hi, per_wave, s);
}

hipError_t launch_expand_level_dev(const DecodeArgs& a, uint32_t level, uint32_t width, uint32_t waves,
                                   hipStream_t s) {
  return launch_expand(a, width, 0u, (int)level, waves, s);
}

hipError_t launch_batch_mark(const BatchArgs& b, hipStream_t s) {
  const uint32_t g = (b.cap + 255) / 256;
  hipLaunchKernelGGL(k_bmark, dim3(g < 1024 ? (g ? g : 1) : 1024), dim3(256), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_batch_close(const BatchArgs& b, uint32_t level, uint32_t width, hipStream_t s) {
  const uint32_t g = (width + 255) / 256;
  if (g == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bclose, dim3(g < 1024 ? g : 1024), dim3(256), 0, s, b, level);
  return hipGetLastError();
}

hipError_t launch_batch_compact(const BatchArgs& b, hipStream_t s) {
  hipLaunchKernelGGL(k_bcompact, dim3(1), dim3(1024), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_batch_gather(const BatchArgs& b, const DecodeArgs& a, hipStream_t s) {
  if (b.cap == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bgather, dim3(b.cap), dim3(256), 0, s, b, a);
  return hipGetLastError();
}

hipError_t launch_persistent(const DecodeArgs& a, uint32_t grid, hipStream_t s) {
  if (a.n_plan == 0) return hipSuccess;
  if (grid == 0) {
    static std::atomic<uint32_t> cache[64];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidValue;
    grid = cache[dev].load(std::memory_order_relaxed);
    if (grid == 0) {
      int cus = 0, per_cu = 0;
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
          hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persist, kPersistThreads, 0) != hipSuccess ||
          cus <= 0)
        return hipErrorUnknown;
      grid = (uint32_t)cus * (uint32_t)(per_cu > 0 ? per_cu : 1);
      cache[dev].store(grid, std::memory_order_relaxed);
    }
  }
  if (grid > a.n_plan) grid = a.n_plan;
  hipLaunchKernelGGL(k_persist, dim3(grid), dim3(kPersistThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_copy(const DecodeArgs& a, const CopyItem* items, uint32_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(n), dim3(256), 0, s, a, items);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  uint64_t g = (n + 255) / 256;
  hipLaunchKernelGGL(k_fill_u32, dim3(g < 4096 ? g : 4096), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed device scratch of the allocation-free seek entry point: one copy per
// device, held from the library's load until the process ends.  Host code
// never passes the array's name to a kernel or a copy (on the host it is a
// stand-in, not a device address): it takes this device's address of the
// array once, with the device current, and uses that.
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

hipError_t static_scratch(void** ptr) {
  static std::mutex mu;
  static void* addr[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> g(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

}  // namespace ace
