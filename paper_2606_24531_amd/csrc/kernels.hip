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
      uint8_t by_rank[4 + 256 + 8];   // k-th present symbol at byte k + 4 (read 8 bytes at a time)
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
        sm.u.b.by_rank[4 + k++] = (uint8_t)s;
        atomicOr(&sm.u.b.starts[cum >> 6], 1ull << (cum & 63));
      }
      cum += f[j];
    }
  }
  wave_sync();
  // ---- slot -> symbol: lane g fills slots 4096/G * g onwards, four slots
  // (one word) at a time.  The symbol of slot t has rank (interval starts at
  // or before t) - 1, so a word's four symbols have ranks prev + c_b, where
  // prev is the rank just before the word and c_b counts the word's starts
  // up to slot b (0..4).  The word is then one byte permute of the 8 rank
  // bytes from prev on: c_b for all four b at once is the word's 4 start
  // bits spread one per byte (a multiply) and prefix-summed across the bytes
  // (a multiply by 0x01010101).  Ranks are stored 4 bytes in, so prev = -1
  // (lane 0; slot 0 always starts an interval) stays in bounds.
  {
    constexpr uint32_t kWpl = 64 / G;  // 64-bit start words per lane
    uint32_t pc = 0;
#pragma unroll
    for (uint32_t q = 0; q < kWpl; q++) pc += __popcll(sm.u.b.starts[kWpl * g + q]);
    uint32_t prev = grp_incl_sum<G>(pc) - pc + 3;  // rank before the lane's first slot, + 4
    uint32_t* out32 = reinterpret_cast<uint32_t*>(sm.sym) + 16 * kWpl * g;
    const uint32_t* br32 = reinterpret_cast<const uint32_t*>(sm.u.b.by_rank);
    if (on) {
#pragma unroll
      for (uint32_t q = 0; q < kWpl; q++) {
        const unsigned long long w = sm.u.b.starts[kWpl * g + q];
#pragma unroll
        for (uint32_t r = 0; r < 16; r++) {
          const uint32_t nib = (uint32_t)(w >> (4 * r)) & 0xFu;
          const uint32_t c = ((nib * 0x00204081u) & 0x01010101u) * 0x01010101u;
          const uint32_t lo = br32[prev >> 2], hi = br32[(prev >> 2) + 1];
          out32[16 * q + r] = __builtin_amdgcn_perm(hi, lo, c + (prev & 3u) * 0x01010101u);
          prev += __popc(nib);
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

// ---------------------------------------------------------------------------
// Entropy coding on the device (the encoder's rANS step, Section 2 and the
// ANS layer of Section 9): one wavefront per stream, output byte for byte
// that of the host encoder.  The frequencies are normalised to 4096 as the
// host does it (f = max(1, floor(c * 4096 / n)), the deficit to the largest
// f, ties to the lower symbol, any excess taken one at a time from the
// largest f > 1); the symbols are coded last to first, lane j holding state
// j (symbols j, j + W, ...), and a step's renormalisation words are numbered
// in the order the host emits them (higher lanes first), so that the words
// read forwards come out in the order the decoder consumes them.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_rans_enc(EncArgs e) {
  __shared__ uint32_t cnt[256];
  __shared__ uint32_t ftab[256], ctab[256];
  const uint32_t i = blockIdx.x, lane = threadIdx.x;
  if (i >= e.n_streams) return;
  const uint32_t n = e.n[i], W = e.W;
  if (n == 0 || e.policy == 2) {
    if (lane == 0) e.out_len[i] = 0;
    return;
  }
  const uint8_t* sym = e.sym + e.sym_off[i];
  for (uint32_t s = lane; s < 256; s += 64) cnt[s] = 0;
  wave_sync();
  for (uint32_t k = lane; k < n; k += 64) atomicAdd(&cnt[ld8(sym + k)], 1u);
  wave_sync();
  // normalisation: lane owns symbols 4 lane .. 4 lane + 3
  uint32_t f[4], sum = 0;
#pragma unroll
  for (uint32_t q = 0; q < 4; q++) {
    const uint64_t c = cnt[4 * lane + q];
    const uint64_t v = c * 4096ull / n;
    f[q] = c ? (v < 1 ? 1u : (uint32_t)v) : 0u;
    sum += f[q];
  }
  sum = uniform(wave_total(sum));
  // the largest f above `floor_` (ties: lower symbol) as f << 8 | (255 - s)
  auto largest = [&](uint32_t floor_) {
    uint32_t key = 0;
#pragma unroll
    for (uint32_t q = 0; q < 4; q++)
      if (f[q] > floor_) key = max(key, (f[q] << 8) | (255u - (4 * lane + q)));
    return uniform(lane63(wave_incl_max(key)));
  };
  if (sum < 4096) {
    const uint32_t best = 255u - (largest(0) & 0xFFu);
    if (best >> 2 == lane) {
#pragma unroll
      for (uint32_t q = 0; q < 4; q++)
        if (q == (best & 3)) f[q] += 4096 - sum;
    }
  }
  for (; sum > 4096; sum--) {
    const uint32_t best = 255u - (largest(1) & 0xFFu);
    if (best >> 2 == lane) {
#pragma unroll
      for (uint32_t q = 0; q < 4; q++)
        if (q == (best & 3)) f[q]--;
    }
  }
  // cumulative frequencies and the table's size
  const uint32_t fl = f[0] + f[1] + f[2] + f[3];
  uint32_t cum = wave_incl_sum(fl, 0) - fl;
  const uint32_t pl = (f[0] != 0) + (f[1] != 0) + (f[2] != 0) + (f[3] != 0);
  uint32_t rank = wave_incl_sum(pl, 0) - pl;
  const uint32_t present = uniform(wave_total(pl));
  const uint32_t tsz = (32 + 2 * present + 3) & ~3u;
#pragma unroll
  for (uint32_t q = 0; q < 4; q++) {
    ftab[4 * lane + q] = f[q];
    ctab[4 * lane + q] = cum;
    cum += f[q];
  }
  wave_sync();
  // code last symbol first; words go to the scratch from its end backwards
  uint16_t* scr = e.scratch + e.scr_off[i];
  uint32_t x = 65536u, emitted = 0;
  const uint32_t steps = (n + W - 1) / W;
  const uint64_t above = lane == 63 ? 0ull : ~0ull << (lane + 1);  // lanes above this one
  for (uint32_t t = steps; t-- > 0;) {
    const uint32_t k = t * W + lane;
    const bool act = lane < W && k < n;
    uint32_t fs = 1, cs = 0;
    if (act) {
      const uint32_t s = ld8(sym + k);
      fs = ftab[s];
      cs = ctab[s];
    }
    const bool emit = act && (uint64_t)x >= ((uint64_t)fs << 20);
    const uint64_t m = __ballot(emit);
    if (emit) {
      const uint32_t r = emitted + (uint32_t)__popcll(m & above);  // the host's word index
      scr[n - 1 - r] = (uint16_t)x;
      x >>= 16;
    }
    emitted += (uint32_t)__popcll(m);
    if (act) x = (x / fs) * 4096u + (x % fs) + cs;
  }
  const uint64_t size = tsz + 4ull * W + 2ull * emitted;
  if (e.policy != 1 && size >= n) {
    if (lane == 0) e.out_len[i] = 0;
    return;
  }
  uint8_t* o = e.out + e.out_off[i];
  // table: presence bitmap (lane l < 32 writes byte l), then f - 1 per
  // present symbol in symbol order, then zero padding to 4 bytes
  const uint32_t bits = (f[0] != 0) | ((f[1] != 0) << 1) | ((f[2] != 0) << 2) | ((f[3] != 0) << 3);
  const uint32_t pair = bits | ((uint32_t)__shfl_xor((int)bits, 1, 64) << 4);  // lanes 2b, 2b + 1
  if (!(lane & 1)) st8(o + (lane >> 1), (uint8_t)pair);
#pragma unroll
  for (uint32_t q = 0; q < 4; q++) {
    if (f[q]) {
      st8(o + 32 + 2 * rank, (uint8_t)(f[q] - 1));
      st8(o + 33 + 2 * rank, (uint8_t)((f[q] - 1) >> 8));
      rank++;
    }
  }
  if (lane < tsz - 32 - 2 * present) st8(o + 32 + 2 * present + lane, 0);
  if (lane < W) {
#pragma unroll
    for (uint32_t b = 0; b < 4; b++) st8(o + tsz + 4 * lane + b, (uint8_t)(x >> (8 * b)));
  }
  uint8_t* wp = o + tsz + 4 * W;
  for (uint32_t w = lane; w < emitted; w += 64) {
    const uint32_t v = scr[n - emitted + w];
    st8(wp + 2 * w, (uint8_t)v);
    st8(wp + 2 * w + 1, (uint8_t)(v >> 8));
  }
  if (lane == 0) e.out_len[i] = (uint32_t)size;
}

// Kernel (a): grid (ceil(n_plan / (64/G)), 3); each wavefront decodes stream
// t of 64/G consecutive plan entries.  LIT goes to lit + plan_index * B, LEN
// to lens + 4 * seq_base and OFF to offs + ow * seq_base; raw streams are
// left in place (the expansion reads them there).  Also records where each
// block's bytes will live.
// Stream t of plan entry i (on: the group has an entry), one group of G lanes.
template <uint32_t G>
__device__ __forceinline__ void rans_entry(const DecodeArgs& a, uint32_t i, bool on, uint32_t t,
                                           RansGroup<G>& sm, uint32_t g, uint32_t h) {
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
  if (rans_decode_group<G>(src, clen, n, a.W, dst, sm, g, h, on) && g == 0) flag(a.err, kErrCorrupt);
  if (a.trace && on && g == 0) {
    a.trace[8ull * i + 2 + 2 * t] = c0;
    a.trace[8ull * i + 3 + 2 * t] = (unsigned long long)wall_clock64();
  }
}

// Kernel (a): grid (x, 3); wavefront x decodes stream y of the 64/G plan
// entries plan_lo + (x + k * gridDim.x) * 64/G + ..., k = 0, 1, ... (one
// pass when the grid covers the plan; a plan whose length is read from
// device memory is covered by striding).  LIT goes to lit + plan_index * B,
// LEN to lens + 4 * seq_base and OFF to offs + ow * seq_base; raw streams
// are left in place (the expansion reads them there).  Also records where
// each block's bytes will live.
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
  for (uint32_t bx = blockIdx.x;; bx += gridDim.x) {
    const uint32_t i = plan_lo + bx * (64 / G) + h;
    const bool on = i < plan_hi;
    if (!__ballot(on)) return;
    rans_entry<G>(a, i, on, t, sm[h], g, h);
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
// Output is then produced in pieces: each literal run and each resolved
// match is cut into 16-byte pieces from its own first byte (the last piece
// shorter; a match repeating a span of 16 bytes or more is cut period by
// period).  A piece is one 16-byte load at any byte alignment (global loads
// and stores take any alignment on this target; a load is moved back when
// the bytes after the piece are not known readable) and one store of
// exactly its bytes; a match whose period is shorter than 16 bytes, or
// whose readable window is too small, is read byte by byte.  Pieces write
// disjoint bytes, so every thread takes kPer of them per round with all
// loads in flight before any store, whatever sequences they belong to.
// Spans that straddle sequences or blocks take the slow path: follow the
// source back until it reaches a literal, a resolved span, an earlier tile
// or an earlier block (each step moves strictly backwards), a run of bytes
// with consecutive sources at a time.
// ---------------------------------------------------------------------------
constexpr uint32_t kPoison = 1u, kSlow = 2u, kPend = 4u, kExt = 8u;
constexpr uint32_t kUnres = kPoison | kSlow | kPend;  // flags of a span without an address
constexpr uint32_t kDepCache = 800;  // dependency lists cached in LDS per block (longer: read from HBM)
constexpr uint32_t kMaxJumps = 12;   // pointer-doubling rounds (chains up to 4096)
constexpr uint32_t kPer = 2;         // output pieces per thread per round

template <uint32_t kThreads>
struct ExpandSmem {
  static constexpr uint32_t kSeq = 2 * kThreads;    // sequences per tile (two per thread)
  static constexpr uint32_t kRound = kPer * kThreads;  // output pieces per round (kPer per thread)
  uint32_t cseq[kRound];  // marks: the sequence whose first piece is each piece of the round (0 = none)
  uint32_t pfx[kSeq];     // index of the sequence's first output piece in the tile
  uint32_t dst[kSeq];     // block-relative start of the sequence
  uint32_t lm[kSeq];      // L | M << 16
  uint32_t lit[kSeq];     // index of the sequence's first literal in the literal stream
  uint32_t dfl[kSeq];     // min(d, 2^24 - 1) | flags << 24
  uint32_t win[kSeq];     // readable bytes around src0: back (0..31) | forward << 5; unresolved: O - block start
  uint32_t ptr[kSeq];     // pending span: span of sequence (ptr >> 16) from offset (ptr & 0xFFFF)
  uint64_t src0[kSeq];    // address of the first byte of a resolved span
  uint32_t deps[kDepCache];
  uint32_t scan[kPer * kThreads / 64 > 32 ? kPer * kThreads / 64 : 32];
};

// A workgroup barrier that orders LDS accesses only: global loads and stores
// still in flight stay in flight (__syncthreads also waits for every one of
// them).  The expansion's barriers guard its LDS tables; its global reads
// never touch bytes written earlier in the same tile.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Whether p holds for any thread of the workgroup (every thread must call
// it; an LDS barrier, with sh[0 .. kThreads/64) as scratch, which the caller
// must not reuse before a later barrier).
template <uint32_t kThreads>
__device__ __forceinline__ bool wg_any(bool p, uint32_t* sh) {
  constexpr uint32_t kW = kThreads / 64;
  const bool w = __ballot(p) != 0;
  if (kW == 1) return w;
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = w ? 1u : 0u;
  lds_barrier();
  uint32_t any = 0;
#pragma unroll
  for (uint32_t q = 0; q < kW; q++) any |= sh[q];
  return any != 0;
}

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
  lds_barrier();
  if (lane == 63) {
#pragma unroll
    for (uint32_t j = 0; j < 4; j++) sh[4 * w + j] = v[j];
  }
  lds_barrier();
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

// Running maximum over N * kThreads values held strided: thread t holds the
// values at positions t + j * kThreads (j < N).  In place,
// v[j] = max(carry, every value at or before its position); returns the
// maximum of all of them and carry.  One barrier (none for one wavefront);
// the caller must order any earlier reads of sh before it.
template <uint32_t kThreads, uint32_t N>
__device__ __forceinline__ uint32_t wg_max_scan_strided(uint32_t (&v)[N], uint32_t carry, uint32_t* sh) {
  constexpr uint32_t kW = kThreads / 64;
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (uint32_t j = 0; j < N; j++) v[j] = wave_incl_max(v[j]);
  uint32_t run = carry;
  if (kW == 1) {
#pragma unroll
    for (uint32_t j = 0; j < N; j++) {
      const uint32_t tot = lane63(v[j]);
      v[j] = max(v[j], run);
      run = max(run, tot);
    }
    return run;
  }
  if (lane == 63) {
#pragma unroll
    for (uint32_t j = 0; j < N; j++) sh[N * w + j] = v[j];
  }
  lds_barrier();
#pragma unroll
  for (uint32_t j = 0; j < N; j++) {
    uint32_t before = run, tot = run;
    for (uint32_t q = 0; q < kW; q++) {
      const uint32_t x = sh[N * q + j];
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

// n / d for n < 2^20 and d >= 1: a reciprocal estimate, then corrected by
// one either way (the estimate is within one of the quotient).
__device__ __forceinline__ uint32_t udiv_small(uint32_t n, uint32_t d) {
  uint32_t q = (uint32_t)((float)n * __builtin_amdgcn_rcpf((float)d));
  if (q * d > n) q--;
  else if ((q + 1) * d <= n) q++;
  return q;
}

// The same for a position p before the end of sequence `from` (sources
// usually lie a few sequences back): steps back 1, 2, 4, ... sequences until
// one starts at or before p, then a binary search within the last step.
__device__ __forceinline__ uint32_t find_seq_before(const uint32_t* sdst, uint32_t from, uint32_t p) {
  if (sdst[from] <= p) return from;
  uint32_t hi = from, step = 1;
  while (true) {
    const uint32_t lo = hi > step ? hi - step : 0u;
    if (sdst[lo] <= p) {
      uint32_t a = lo, b = hi;  // sdst[a] <= p < sdst[b]
      while (b - a > 1) {
        const uint32_t mid = (a + b) >> 1;
        if (sdst[mid] <= p) a = mid; else b = mid;
      }
      return a;
    }
    hi = lo;
    step <<= 1;
  }
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

// Source offset of a sequence without a resolved address, relative to the
// block start, as a signed 32-bit value (kOrelFar: too far back; then it is
// read back from the offset stream).
constexpr uint32_t kOrelFar = 0x80000000u;
__device__ __forceinline__ uint32_t orel_pack(uint64_t o, uint64_t bs) {
  const int64_t r = (int64_t)(o - bs);
  return r > -(int64_t)0x7FFFFFFF && r < (int64_t)0x7FFFFFFF ? (uint32_t)(int32_t)r : kOrelFar;
}

// Slow path: the address of the byte at block-relative p, following sources
// back to a literal, a resolved span, an earlier tile of this block or an
// earlier block (each step moves strictly backwards, so the walk ends), and
// in run the number of bytes from p on whose sources lie consecutively from
// that address (at least 1: the walk stops narrowing it at segment ends, a
// period's wrap, the earlier tiles' end and the current block's start).
// Null when the bytes are to be written as zeros (a failed format rule, or an
// earlier block that was never published).  ext: the address lies in an
// earlier block.  Reads LDS and (outside whole-archive decodes, or for
// offsets too far back) the location table and the offset stream.
template <uint32_t kThreads>
__device__ const uint8_t* resolve_run(const DecodeArgs& a, const ExpandSmem<kThreads>& sm, const BlockCtx& c,
                                      uint32_t s, uint32_t p, uint32_t& run, bool& ext) {
  uint32_t lim = 0xFFFFFFFFu;
  ext = false;
  for (;;) {
    const uint32_t fl = sm.dfl[s] >> 24;
    const uint32_t r = p - sm.dst[s];
    const uint32_t Ls = sm.lm[s] & 0xFFFFu, Ms = sm.lm[s] >> 16;
    if (fl & kPoison) {
      run = min(lim, Ls + Ms > r ? Ls + Ms - r : 1u);
      return nullptr;
    }
    if (r < Ls) {
      run = min(lim, Ls - r);
      return c.lit + sm.lit[s] + r;
    }
    const uint32_t ii = r - Ls, d = sm.dfl[s] & 0xFFFFFFu;
    const uint32_t im = ii < d ? ii : ii - d * udiv_small(ii, d);  // ii < 2^16
    lim = min(lim, Ms > d ? min(Ms - ii, d - im) : Ms - ii);
    if (!(fl & kUnres)) {
      run = lim;
      ext = (fl & kExt) != 0;
      return reinterpret_cast<const uint8_t*>(sm.src0[s] + im);
    }
    // the source offset, kept beside the sequence (read back from the token
    // stream when too far back for 32 bits)
    const uint32_t orel = sm.win[s];
    const uint32_t k = c.t0 + s;
    const uint64_t o = orel != kOrelFar ? c.bs + (uint64_t)(int64_t)(int32_t)orel
                       : c.ow == 4 ? (uint64_t)ld32(c.offs + 4ull * k) : ld64(c.offs + 8ull * k);
    const uint64_t src = o + im;
    if (src < c.bs) {
      if (!c.ext_ok) {
        run = 1;
        return nullptr;
      }
      const uint64_t blk = blk_of(a, src);
      const uint64_t room = a.loc_linear ? c.bs - src : (blk + 1) * a.B - src;  // contiguous bytes there
      run = (uint32_t)min((uint64_t)lim, room);
      ext = true;
      return reinterpret_cast<const uint8_t*>(blk_loc(a, blk)) + (src - blk * a.B);
    }
    const uint32_t q = (uint32_t)(src - c.bs);
    if (q < c.d0) {
      run = min(lim, c.d0 - q);
      return c.out + q;
    }
    s = find_seq_before(sm.dst, s, q);  // the source lies before this sequence
    p = q;
  }
}

// The slot holding slow byte u of the tile: slot k's slow bytes (its match
// bytes, numbered in sequence order) end at sm.ptr[k].
template <uint32_t kThreads>
__device__ __forceinline__ uint32_t slow_slot(const ExpandSmem<kThreads>& sm, const BlockCtx& c, uint32_t u) {
  uint32_t lo = 0, hi = c.cnt;  // first slot whose slow-byte end exceeds u
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (sm.ptr[mid] > u) hi = mid; else lo = mid + 1;
  }
  return lo;
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

// The 16 bytes x moved down by s bytes (byte s becomes byte 0; zeros come
// in at the top), 0 <= s < 16.  Branch-free: dword selects, then a funnel
// shift.
__device__ __forceinline__ uint32_t pick4(const uint32_t (&y)[8], uint32_t i, uint32_t q) {
  return q == 0 ? y[i] : q == 1 ? y[i + 1] : q == 2 ? y[i + 2] : y[i + 3];
}
__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t b) {  // b in 0..24 step 8
  return __builtin_amdgcn_alignbyte(hi, lo, b >> 3);  // bytes b/8.. of hi:lo
}
__device__ __forceinline__ void shift_down16(uint32_t (&x)[4], uint32_t s) {
  const uint32_t q = s >> 2, b = 8 * (s & 3);
  const uint32_t y[8] = {x[0], x[1], x[2], x[3], 0u, 0u, 0u, 0u};
  uint32_t z[5];
#pragma unroll
  for (uint32_t i = 0; i < 5; i++) z[i] = pick4(y, i < 4 ? i : 4, q);
#pragma unroll
  for (uint32_t i = 0; i < 4; i++) x[i] = funnel(z[i + 1], z[i], b);
}
typedef uint64_t u64_a1 __attribute__((aligned(1)));
typedef uint32_t u32_a1 __attribute__((aligned(1)));
typedef uint16_t u16_a1 __attribute__((aligned(1)));
// Writes bytes [0, len) of w (len <= 16) at any byte address, nothing else.
__device__ __forceinline__ void store_bytes(uint8_t* p, const uint32_t (&w)[4], uint32_t len) {
  if (len == 16) {
    st16u(p, make_uint4(w[0], w[1], w[2], w[3]));
    return;
  }
  uint32_t x0 = w[0], x1 = w[1], x2 = w[2], x3 = w[3], o = 0;
  if (len & 8) {
    *reinterpret_cast<ACE_GLOBAL u64_a1*>(gp(p)) = (uint64_t)x0 | ((uint64_t)x1 << 32);
    x0 = x2;
    x1 = x3;
    o = 8;
  }
  if (len & 4) {
    *reinterpret_cast<ACE_GLOBAL u32_a1*>(gp(p + o)) = x0;
    x0 = x1;
    o += 4;
  }
  if (len & 2) {
    *reinterpret_cast<ACE_GLOBAL u16_a1*>(gp(p + o)) = (uint16_t)x0;
    x0 >>= 16;
    o += 2;
  }
  if (len & 1) st8(p + o, (uint8_t)x0);
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

// Output pieces of a match of m bytes (m < 2^16) whose byte i is span byte
// i mod d: a match that repeats its span (m > d) with d >= 16 is cut period
// by period, each period into 16-byte pieces from its start; any other match
// into 16-byte pieces from its first byte.
__device__ __forceinline__ uint32_t match_pieces(uint32_t m, uint32_t d) {
  if (m <= d || d < 16) return (m + 15) >> 4;
  const uint32_t q = udiv_small(m, d);
  return q * ((d + 15) >> 4) + ((m - q * d + 15) >> 4);
}

// Expands plan entry i with kThreads threads.  Sources in earlier blocks must
// be complete and visible (unless ext_ok is false, after a timed-out wait).
template <uint32_t kThreads>
__device__ __forceinline__ void expand_block(const DecodeArgs& a, uint32_t i, ExpandSmem<kThreads>& sm,
                                             bool ext_ok = true) {
  constexpr uint32_t kSeq = ExpandSmem<kThreads>::kSeq, kRound = ExpandSmem<kThreads>::kRound;
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
  const bool cached = dep_cnt <= kDepCache;
  uint32_t carry_pos = 0, carry_lit = 0, n_ext = 0;
  bool bad = false;
  // the piece marks start cleared (each thread clears the entries it later
  // reads, right after reading them), ordered before the first marks by the
  // barriers of the token phase
#pragma unroll
  for (uint32_t j = 0; j < kPer; j++) sm.cseq[tid + j * kThreads] = 0;
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
      // a span without an address keeps its source offset here instead
      sm.win[slot] = (fl & (kSlow | kPend)) ? orel_pack(O[h], c.bs) : win;
      sm.src0[slot] = src0;
    }
    lds_barrier();
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
      sm.win[slot] = fl ? orel_pack(O[h], c.bs) : win;
      fl_h[h] = fl;
    }
    // ---- pointer doubling
    for (uint32_t round = 0;; round++) {
      const bool pend = (fl_h[0] | fl_h[1]) & kPend;
      if (!wg_any<kThreads>(pend, sm.scan)) break;
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
      lds_barrier();
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
    const uint64_t d1w = (uint64_t)carry_pos + tp;
    const uint32_t d1 = d1w < c.blen ? (uint32_t)d1w : c.blen;
    // Output pieces: every sequence's literal run and its match (unless the
    // match is slow) are cut into pieces of 16 bytes from their own start,
    // the last one shorter; a poisoned sequence's bytes (clipped to the
    // tile) are pieces of zeros.  Pieces write disjoint bytes, so they are
    // spread over the threads in any order.  Slow sequences' match bytes
    // are numbered for the slow pass: slot k's slow bytes end at sm.ptr[k]
    // (the pointers are no longer needed), its pieces start at sm.pfx[k].
    uint32_t n_slow = 0, n_piece = 0;
    {
      uint32_t np[2];
#pragma unroll
      for (uint32_t h = 0; h < 2; h++) {
        const uint32_t slot = tid + h * kThreads;
        uint32_t n = 0;
        if (slot < c.cnt) {
          if (fl_h[h] & kPoison) {
            const uint32_t ds = pos_h[h];
            const uint64_t e = (uint64_t)ds + L[h] + M[h];
            n = ds < d1 ? ((e < d1 ? (uint32_t)e : d1) - ds + 15) >> 4 : 0u;
          } else {
            n = ((L[h] + 15) >> 4) + ((fl_h[h] & kSlow) ? 0u : match_pieces(M[h], sm.dfl[slot] & 0xFFFFFFu));
          }
        }
        np[h] = n;
      }
      uint32_t cv[4] = {(fl_h[0] & kSlow) ? M[0] : 0u, np[0], (fl_h[1] & kSlow) ? M[1] : 0u, np[1]}, ct[4];
      wg_scan4<kThreads>(cv, ct, sm.scan);
      sm.ptr[tid] = cv[0];
      sm.ptr[tid + kThreads] = ct[0] + cv[2];
      sm.pfx[tid] = cv[1] - np[0];
      sm.pfx[tid + kThreads] = ct[1] + cv[3] - np[1];
      n_slow = ct[0] + ct[2];
      n_piece = ct[1] + ct[3];
      lds_barrier();
    }
    // ---- pieces, kPer per thread per round: thread t takes pieces
    // t + j * kThreads of the round.  Each sequence marks its first piece;
    // a running maximum over the round's pieces gives every piece its
    // sequence.  All of a thread's loads are issued before any is stored.
    uint32_t carry = 0;  // the last sequence marked in earlier rounds
    for (uint32_t p0 = 0; p0 < n_piece; p0 += kRound) {
#pragma unroll
      for (uint32_t h = 0; h < 2; h++) {
        const uint32_t slot = tid + h * kThreads;
        if (slot < c.cnt) {
          const uint32_t f = sm.pfx[slot];
          const uint32_t nxt = slot + 1 < c.cnt ? sm.pfx[slot + 1] : n_piece;
          if (nxt > f && f >= p0 && f < p0 + kRound) sm.cseq[f - p0] = slot;
        }
      }
      lds_barrier();
      uint32_t sqv[kPer];
#pragma unroll
      for (uint32_t j = 0; j < kPer; j++) {
        sqv[j] = sm.cseq[tid + j * kThreads];
        sm.cseq[tid + j * kThreads] = 0;
      }
      carry = wg_max_scan_strided<kThreads, kPer>(sqv, carry, sm.scan);
      uint4 v1[kPer];
      uint32_t dsto[kPer], len[kPer], sh1[kPer];
#pragma unroll
      for (uint32_t j = 0; j < kPer; j++) {
        const uint32_t p = p0 + tid + j * kThreads;
        const bool on = p < n_piece;
        const uint32_t sq = sqv[j] < c.cnt ? sqv[j] : c.cnt - 1;
        const uint32_t pf = sm.pfx[sq], ds = sm.dst[sq], lmv = sm.lm[sq], litv = sm.lit[sq];
        const uint32_t dfl = sm.dfl[sq], wn = sm.win[sq];
        const uint64_t s0 = sm.src0[sq];
        const uint32_t Ls = lmv & 0xFFFFu, Ms = lmv >> 16, fl = dfl >> 24, dist = dfl & 0xFFFFFFu;
        const uint32_t k = on ? p - pf : 0u;
        const uint32_t pl = (Ls + 15) >> 4;
        // the piece: output offset, length, and where its bytes come from
        const uint8_t* A1 = c.lit;  // readable: the literal stream has slack around it
        uint32_t off, r, s1 = 0, at = 0;
        const bool zero = !on || (fl & kPoison);
        if ((fl & kPoison) || k < pl) {
          off = 16 * k;
          const uint32_t tot = (fl & kPoison) ? (d1 - ds < Ls + Ms ? d1 - ds : Ls + Ms) : Ls;
          r = tot - off < 16 ? tot - off : 16;
          A1 = c.lit + litv + off;
          dsto[j] = ds + off;
        } else {
          // match byte i reads span byte i mod d: a match that repeats its
          // span with a period of 16 bytes or more is cut period by period
          // (no piece crosses a period's end); a shorter period goes byte
          // by byte below
          const uint32_t kk = k - pl;
          if (Ms > dist && dist >= 16) {
            const uint32_t ppp = (dist + 15) >> 4, q = udiv_small(kk, ppp);
            at = 16 * (kk - q * ppp);
            off = q * dist + at;
            const uint32_t rest = dist - at < Ms - off ? dist - at : Ms - off;
            r = rest < 16 ? rest : 16;
          } else {
            off = at = 16 * kk;
            r = Ms - off < 16 ? Ms - off : 16;
          }
          dsto[j] = ds + Ls + off;
          // readable bytes around the span start: back (<= 31), forward
          const uint32_t back = wn & 31u, fwd = wn >> 5;
          const uint32_t need = at + 16 > fwd ? at + 16 - fwd : 0u;  // shift the load back this far
          s1 = need;
          A1 = reinterpret_cast<const uint8_t*>(s0 + at - need);
          if (need > back + at || (Ms > dist && dist < 16)) {
            // a window too small for a 16-byte load, or a period shorter
            // than a piece: this piece goes byte by byte below
            s1 = 0xFFu;
            A1 = c.lit;
          }
        }
        len[j] = on ? r : 0u;
        sh1[j] = zero ? 0x100u : s1;  // 0x100: zeros
        v1[j] = ld16u(zero || s1 == 0xFFu ? c.lit : A1);
        if (s1 == 0xFFu && !zero) {
          // byte by byte (rare): span byte (off + i) mod d for each piece byte
          uint32_t w[4] = {0, 0, 0, 0};
          uint32_t ii = Ms > dist ? off % dist : off;
#pragma unroll
          for (uint32_t b2 = 0; b2 < 16; b2++) {
            if (b2 < r) w[b2 >> 2] |= (uint32_t)ld8(reinterpret_cast<const uint8_t*>(s0 + ii)) << (8 * (b2 & 3));
            ii = (Ms > dist && ii + 1 == dist) ? 0u : ii + 1;
          }
          v1[j] = make_uint4(w[0], w[1], w[2], w[3]);
          sh1[j] = 0;
        }
      }
      // assemble and store: the load shifted down by sh1 (or zeros);
      // exactly len bytes written
#pragma unroll
      for (uint32_t j = 0; j < kPer; j++) {
        if (!len[j]) continue;
        uint32_t w[4] = {v1[j].x, v1[j].y, v1[j].z, v1[j].w};
        if (sh1[j] == 0x100u) {
          w[0] = w[1] = w[2] = w[3] = 0u;
        } else if (sh1[j] != 0) {  // a load moved back (rare): bytes to line up
          shift_down16(w, sh1[j]);
        }
        store_bytes(c.out + dsto[j], w, len[j]);
      }
      lds_barrier();  // the marks of the next round are written after every read of this one
    }
    // ---- slow pass: the match bytes of slow sequences (spans that straddle
    // sequences, tiles or non-adjacent blocks), each thread an equal share of
    // consecutive ones, followed back to their origin (never to this tile's
    // output) a run of consecutive sources at a time
    if (n_slow) {
      const uint32_t per = (n_slow + kThreads - 1) / kThreads;
      uint32_t u = tid * per;
      const uint32_t u1 = min(u + per, n_slow);
      uint32_t k = u < u1 ? slow_slot<kThreads>(sm, c, u) : 0u;
      while (u < u1) {
        const uint32_t Mk = sm.lm[k] >> 16, end_k = sm.ptr[k];
        const uint32_t p = sm.dst[k] + (sm.lm[k] & 0xFFFFu) + (u - (end_k - Mk));
        uint32_t run;
        bool ext;
        const uint8_t* q = resolve_run<kThreads>(a, sm, c, k, p, run, ext);
        const uint32_t n = min(min(run, u1 - u), end_k - u);
        if (ext) n_ext += n;
        for (uint32_t i = 0; i < n; i += 4) {
          uint8_t v[4];
#pragma unroll
          for (uint32_t j = 0; j < 4; j++) v[j] = (q && i + j < n) ? ld8(q + i + j) : (uint8_t)0;
#pragma unroll
          for (uint32_t j = 0; j < 4; j++)
            if (i + j < n) st8(c.out + p + i + j, v[j]);
        }
        u += n;
        while (u < u1 && sm.ptr[k] <= u) k++;  // on to the next slow slot
      }
    }
    // the next tile reads this tile's output and rewrites the tables
    if (t0 + kSeq < n_seq) __syncthreads();
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
  lds_barrier();
  if ((tid & 63) == 0) sm.scan[tid >> 6] = n_ext;
  lds_barrier();
  if (tid == 0) {
    uint32_t sum = 0;
    for (uint32_t w = 0; w < kThreads / 64; w++) sum += sm.scan[w];
    if (sum) atomicAdd(a.ext_bytes + (b & 15), (unsigned long long)sum);
  }
}

template <uint32_t kThreads>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kThreads == 128 ? 6 : 4))) void k_expand(
    DecodeArgs a, uint32_t plan_lo, int level) {
  __shared__ ExpandSmem<kThreads> sm;
  // host-planned: one block per workgroup; device-planned: the level's plan
  // range from device memory, strided over the grid (one call site, so the
  // expansion is inlined)
  const bool host = level < 0;
  const uint32_t first = (host ? plan_lo : a.lvl_dev[level]) + blockIdx.x;
  const uint32_t end = host ? first + 1 : a.lvl_dev[level + 1];
  const uint32_t stride = host ? 1u : gridDim.x;
  for (uint32_t i = first; i < end; i += stride) {
    const unsigned long long c0 = a.trace ? (unsigned long long)wall_clock64() : 0ull;
    expand_block<kThreads>(a, i, sm);
    if (a.trace && threadIdx.x == 0) {
      a.trace[8ull * i] = c0;
      a.trace[8ull * i + 1] = (unsigned long long)wall_clock64();
    }
    if (i + stride < end) lds_barrier();  // every thread done with this block's LDS tables
  }
}

// ---------------------------------------------------------------------------
// Kernel (c): one persistent launch expands a whole plan, level by level
// (the entropy layer of every planned block is decoded by kernel (a) just
// before it), with device-side counters.
//
// A level's blocks are dealt into kPersistSlices slices (block j of the level
// to slice j mod kPersistSlices), each with its own claim counter on its own
// cache line.  Workgroup w claims from slice w mod kPersistSlices (its home:
// with workgroups dealt round-robin over the XCDs, one slice per XCD), and
// once that is empty from the others in turn, so no single address takes
// every claim.  The next claim on the home slice is issued before the claimed
// block's expansion and its result used after it, which hides the atomic's
// round trip.  When no slice has blocks left, the workgroup adds the count it
// expanded to the level's finished count (one atomic per workgroup and
// level); the workgroup whose add completes the level raises the count of
// finished levels held in kPersistReplicas copies, one per 128-byte line, and
// each workgroup polls the copy w mod kPersistReplicas until it passes the
// level, so idle polling is spread over many lines.  Only workgroups
// 0 .. size-1 claim from a level of `size` blocks (the others go straight to
// the wait, so a small level is not probed by the whole grid).  Empty levels
// are skipped.  A block's dependencies all sit at lower levels, so every block
// expanded finds its sources complete.  A workgroup waits only after every
// block of the level is claimed, i.e. held by a running workgroup: the launch
// needs no co-residency, and drains when it shares the device.
//
// Visibility across workgroups: every wave of a workgroup issues an
// agent-scope release fence (its stores complete, this XCD's L2 written
// back) before the barrier that precedes the workgroup's finished-count add;
// the copies are raised by atomic max after that add.  A waiting workgroup
// polls with agent-scope atomic loads; a workgroup that claims a block of the
// next level issues an agent-scope acquire fence in every wave before it
// reads lower levels' bytes.
//
// Every wait is bounded by a count of idle polls (not by a clock).  An
// expired wait flags kErrTimeout and the workgroup stops waiting from then
// on, as does every workgroup that sees that flag (checked every 256 idle
// polls); expansions then no longer read earlier blocks, so the launch always
// drains (its output is then not valid, and ace_check reports the timeout).
// ---------------------------------------------------------------------------
// The XCD (accelerator complex die) this wave runs on: the XCC_ID hardware
// register, bits 3:0.
__device__ __forceinline__ uint32_t xcc_id() {
  return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (kMaxXcc - 1);
}

constexpr uint32_t kPersistThreads = 128;
constexpr uint32_t kNoItem = 0xffffffffu;

// A counter shared across workgroups, read at agent scope.
__device__ __forceinline__ uint32_t coherent_u32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Blocks of a level of `size` blocks in slice r.
__device__ __forceinline__ uint32_t slice_size(uint32_t size, uint32_t r) {
  return size > r ? (size - 1 - r) / kPersistSlices + 1 : 0u;
}

// A claim from any slice with blocks left, starting at slice `first`
// (thread 0 only): the plan entry, or kNoItem when every slice is empty.
__device__ uint32_t claim_any(const DecodeArgs& a, uint32_t lvl, uint32_t lo, uint32_t size, uint32_t first) {
  for (uint32_t k = 0; k < kPersistSlices; k++) {
    const uint32_t r = (first + k) % kPersistSlices, n_r = slice_size(size, r);
    if (n_r == 0) continue;
    uint32_t* c = a.lvl_claim + (uint64_t)r * a.lvl_row + lvl;
    if (coherent_u32(c) >= n_r) continue;
    const uint32_t t = atomicAdd(c, 1u);
    if (t < n_r) return lo + r + t * kPersistSlices;
  }
  return kNoItem;
}

__global__ __launch_bounds__(kPersistThreads) __attribute__((amdgpu_waves_per_eu(5))) void k_persist(DecodeArgs a) {
  __shared__ ExpandSmem<kPersistThreads> sm;
  __shared__ uint32_t sh_item[2], sh_give_up;
  const uint32_t tid = threadIdx.x, home = blockIdx.x % kPersistSlices;
  uint32_t* seen = a.lvl_seen + (blockIdx.x % kPersistReplicas) * kPersistLine;
  bool give_up = false;  // thread 0's view, broadcast after every wait
  for (uint32_t lvl = 0; lvl < a.n_lvl; lvl++) {
    const uint32_t lo = a.lvl_dev[lvl], size = a.lvl_dev[lvl + 1] - lo;
    if (size == 0) continue;
    // workgroups 0 .. size-1 take part (all of them when the level has at
    // least as many blocks as the grid); workgroups are dispatched in index
    // order, so every one taking part is running while any other waits
    uint32_t mine = 0;
    if (blockIdx.x < size) {
      const uint32_t n_home = slice_size(size, home);
      uint32_t* home_claim = a.lvl_claim + (uint64_t)home * a.lvl_row + lvl;
      unsigned long long* xc = a.lvl_xcd + (uint64_t)lvl * 2 * kMaxXcc + xcc_id();
      if (tid == 0) {
        sh_item[0] = claim_any(a, lvl, lo, size, home);
        // expanding on this XCD from now on (before any of this level's stores)
        if (sh_item[0] != kNoItem) atomicAdd(xc, 1ull);
      }
      __syncthreads();
      uint32_t item = sh_item[0], par = 0;
      // the levels below are complete: make their bytes visible here (only
      // workgroups with blocks to expand pay for the cache invalidation)
      if (item != kNoItem) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      while (item != kNoItem) {
        uint32_t next = kNoItem;
        if (tid == 0) next = atomicAdd(home_claim, 1u);  // result used after the expansion
        const unsigned long long c0 = a.trace ? (unsigned long long)wall_clock64() : 0ull;
        expand_block<kPersistThreads>(a, item, sm, !give_up);
        if (a.trace && tid == 0) {
          a.trace[8ull * item] = c0;
          a.trace[8ull * item + 1] = (unsigned long long)wall_clock64();
        }
        mine++;
        if (tid == 0)
          sh_item[par ^ 1] = next < n_home ? lo + home + next * kPersistSlices : claim_any(a, lvl, lo, size, home + 1);
        lds_barrier();  // every thread done with this block's LDS tables; next item visible
        par ^= 1;
        item = sh_item[par];
      }
      if (mine) {
        // this workgroup's stores have reached its XCD's L2.  Leaving, it
        // adds its blocks to the XCD's running count; the workgroup that
        // leaves the XCD with none expanding writes that L2 back once (an
        // agent-scope release, covering every block counted so far) and
        // raises the XCD's written-back count to the running count, adding
        // what it raised to the level's finished count.  A level is
        // complete once every XCD holding its bytes has written them back.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        if (tid < kPersistReplicas) {  // wave 0: lane r raises copy r
          uint32_t add = 0, prev = 0;
          if (tid == 0) {
            const unsigned long long old = atomicAdd(xc, ((unsigned long long)mine << 32) - 1ull);
            if ((uint32_t)old == 1u) {
              __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
              const unsigned long long total = (old >> 32) + mine;
              const unsigned long long was = atomicMax(xc + kMaxXcc, total);
              add = total > was ? (uint32_t)(total - was) : 0u;
              if (add) prev = atomicAdd(a.lvl_done + lvl, add);
            }
          }
          add = __shfl(add, 0);
          prev = __shfl(prev, 0);
          if (add && prev + add == size) {
            // no fence here: every XCD holding the level's bytes wrote them
            // back before its add, and this raise is issued after the add
            // that returned the level complete
            __hip_atomic_fetch_max(a.lvl_seen + tid * kPersistLine, lvl + 1, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
          }
          __builtin_amdgcn_wave_barrier();  // the wave's raises come before lane 0's wait
        }
      }
    }
    if (tid == 0) {
      uint32_t idle = 0;
      while (!give_up && coherent_u32(seen) <= lvl) {
        if (idle < 16) __builtin_amdgcn_s_sleep(4);
        else __builtin_amdgcn_s_sleep(32);
        ++idle;
        if (idle > a.max_polls || ((idle & 255u) == 0 && (coherent_u32(a.err) & kErrTimeout))) {
          flag(a.err, kErrTimeout);
          give_up = true;
        }
      }
      sh_give_up = give_up ? 1u : 0u;
    }
    __syncthreads();
    give_up = sh_give_up != 0;
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

// One wavefront per block of the level (lanes over its dependency list).
__global__ __launch_bounds__(256) void k_bclose(BatchArgs b, uint32_t level) {
  const uint32_t lane = threadIdx.x & 63, wpg = blockDim.x >> 6;
  const uint32_t j0 = b.lstart[level], j1 = b.lstart[level + 1];
  for (uint32_t j = j0 + blockIdx.x * wpg + (threadIdx.x >> 6); j < j1; j += gridDim.x * wpg) {
    const uint32_t blk = b.order[j];
    if (!b.need[blk]) continue;  // uniform over the wavefront
    const uint8_t* be = b.arch + kHdr + (uint64_t)kBlk * blk;
    const uint32_t dep_off = ld32(be + 20), dep_cnt = ld32(be + 24);
    const uint32_t* deps = reinterpret_cast<const uint32_t*>(b.arch + kHdr + (uint64_t)kBlk * b.n_blocks) + dep_off;
    for (uint32_t k = lane; k < dep_cnt; k += 64) {
      const uint32_t d = deps[k];
      if (!b.pin[d]) b.need[d] = 1;
    }
  }
}

// Compaction of the needed blocks, in level order, into the plan: chunks of
// kCompactChunk positions of `order`.  (1) each workgroup counts its chunk's
// needed blocks and their sequences; (2) one workgroup scans the chunk
// totals; (3) each workgroup writes its chunk's plan entries at their scanned
// positions, the level boundaries of the levels that start in it, and
// (last chunk) the plan length.
constexpr uint32_t kCompactChunk = 1024;

__device__ __forceinline__ void need_fields(const BatchArgs& b, uint32_t j, uint32_t& blk, uint32_t& f,
                                            uint32_t& ns) {
  blk = 0;
  f = 0;
  ns = 0;
  if (j < b.n_blocks) {
    blk = b.order[j];
    f = b.need[blk] ? 1u : 0u;
    ns = f ? ld32(b.arch + kHdr + (uint64_t)kBlk * blk + 12) : 0u;
  }
}

// Workgroup sums (kCompactChunk threads) of f and ns; exclusive prefixes of
// both in oc / os for the calling thread.
__device__ __forceinline__ void chunk_scan(uint32_t f, uint32_t ns, uint32_t& oc, uint32_t& os, uint32_t& tc,
                                           uint32_t& ts) {
  __shared__ uint32_t sh_cnt[kCompactChunk / 64], sh_seq[kCompactChunk / 64];
  const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t ic = wave_incl_sum(f, lane), is = wave_incl_sum(ns, lane);
  if (lane == 63) {
    sh_cnt[w] = ic;
    sh_seq[w] = is;
  }
  __syncthreads();
  oc = ic - f;
  os = is - ns;
  tc = ts = 0;
  for (uint32_t k = 0; k < kCompactChunk / 64; k++) {
    if (k < w) {
      oc += sh_cnt[k];
      os += sh_seq[k];
    }
    tc += sh_cnt[k];
    ts += sh_seq[k];
  }
}

__global__ __launch_bounds__(kCompactChunk) void k_bcount(BatchArgs b) {
  uint32_t blk, f, ns, oc, os, tc, ts;
  need_fields(b, blockIdx.x * kCompactChunk + threadIdx.x, blk, f, ns);
  chunk_scan(f, ns, oc, os, tc, ts);
  if (threadIdx.x == 0) {
    b.chunk_cnt[blockIdx.x] = tc;
    b.chunk_seq[blockIdx.x] = ts;
  }
}

// One workgroup: exclusive scans of the chunk totals, in place; the grand
// totals after the last chunk.
__global__ __launch_bounds__(1024) void k_bscan(BatchArgs b, uint32_t n_chunks) {
  __shared__ uint32_t sh_c[16], sh_s[16], base_c, base_s;
  const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) base_c = base_s = 0;
  __syncthreads();
  for (uint32_t c0 = 0; c0 <= n_chunks; c0 += 1024) {
    const uint32_t c = c0 + tid;
    const uint32_t vc = c < n_chunks ? b.chunk_cnt[c] : 0u, vs = c < n_chunks ? b.chunk_seq[c] : 0u;
    const uint32_t ic = wave_incl_sum(vc, lane), is = wave_incl_sum(vs, lane);
    if (lane == 63) {
      sh_c[w] = ic;
      sh_s[w] = is;
    }
    __syncthreads();
    uint32_t oc = base_c + ic - vc, os = base_s + is - vs, tc = 0, ts = 0;
    for (uint32_t k = 0; k < 16; k++) {
      if (k < w) {
        oc += sh_c[k];
        os += sh_s[k];
      }
      tc += sh_c[k];
      ts += sh_s[k];
    }
    if (c <= n_chunks) {
      b.chunk_cnt[c] = oc;  // chunk n_chunks receives the grand totals
      b.chunk_seq[c] = os;
    }
    __syncthreads();
    if (tid == 0) {
      base_c += tc;
      base_s += ts;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kCompactChunk) void k_bwrite(BatchArgs b, uint32_t n_chunks) {
  const uint32_t j = blockIdx.x * kCompactChunk + threadIdx.x;
  uint32_t blk, f, ns, oc, os, tc, ts;
  need_fields(b, j, blk, f, ns);
  chunk_scan(f, ns, oc, os, tc, ts);
  const uint32_t pos = b.chunk_cnt[blockIdx.x] + oc, seq = b.chunk_seq[blockIdx.x] + os;
  if (j < b.n_blocks) {
    b.pre[j] = pos;
    // the first position of a level: that level's plan start
    const uint8_t* be = b.arch + kHdr + (uint64_t)kBlk * blk;
    const uint32_t lv = ld32(be + 16);
    if (b.lstart[lv] == j) b.lvl_dev[lv] = pos;
  }
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
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const uint32_t total = b.chunk_cnt[n_chunks];
    b.lvl_dev[b.depth] = total;
    *b.n_plan_dev = total;
  }
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

__global__ void k_put_range(uint64_t* desc, uint64_t d_out, uint64_t lo, uint64_t hi) {
  const uint64_t v[5] = {1, d_out, lo, hi, 0};
  if (threadIdx.x < 5) desc[threadIdx.x] = v[threadIdx.x];
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint64_t n) {
  for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < n;
       j += (uint64_t)gridDim.x * blockDim.x)
    p[j] = v;
}

}  // namespace

// Grid caps of launches whose plan length is read on the device.
constexpr uint32_t kStrideGridRans = 4096, kStrideGridExpand = 2048;

// Entropy launch over plan entries [lo, hi), or (lv_lo >= 0) over the plan
// range of levels [lv_lo, lv_hi) read from device memory, with hi - lo
// entries of capacity.
static hipError_t launch_rans_any(const DecodeArgs& a, uint32_t lo, uint32_t hi, int lv_lo, int lv_hi,
                                  uint32_t per_wave, hipStream_t s) {
  if (hi <= lo) return hipSuccess;
  const uint32_t n = hi - lo;
  if (per_wave == 0) per_wave = a.W <= 32 ? 2 : 1;
  const bool two = per_wave == 2 && a.W <= 32;
  uint32_t grid = two ? (n + 1) / 2 : n;
  // a plan whose length is read on the device is covered by striding over a
  // grid the device holds at once, not by one wavefront per possible entry
  const bool dev = lv_lo >= 0 || a.n_plan_dev;
  if (dev && grid > kStrideGridRans) grid = kStrideGridRans;
  if (two)
    hipLaunchKernelGGL(k_rans<32>, dim3(grid, 3), dim3(64), 0, s, a, lo, hi, lv_lo, lv_hi);
  else
    hipLaunchKernelGGL(k_rans<64>, dim3(grid, 3), dim3(64), 0, s, a, lo, hi, lv_lo, lv_hi);
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

hipError_t launch_rans_encode(const EncArgs& e, hipStream_t s) {
  if (e.n_streams == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rans_enc, dim3(e.n_streams), dim3(64), 0, s, e);
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
  // strided over at most as many workgroups as the device holds at once
  const uint32_t r4 = expand4_resident();
  const uint32_t cap = r4 ? 2 * r4 : kStrideGridExpand;
  return launch_expand(a, width < cap ? width : cap, 0u, (int)level, waves, s);
}

hipError_t launch_batch_mark(const BatchArgs& b, hipStream_t s) {
  const uint32_t g = (b.cap + 255) / 256;
  hipLaunchKernelGGL(k_bmark, dim3(g < 1024 ? (g ? g : 1) : 1024), dim3(256), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_batch_close(const BatchArgs& b, uint32_t level, uint32_t width, hipStream_t s) {
  const uint32_t g = (width + 3) / 4;  // four wavefronts per workgroup, one per block
  if (g == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bclose, dim3(g < 4096 ? g : 4096), dim3(256), 0, s, b, level);
  return hipGetLastError();
}

uint32_t batch_compact_chunks(uint32_t n_blocks) { return (n_blocks + kCompactChunk - 1) / kCompactChunk; }

hipError_t launch_batch_compact(const BatchArgs& b, hipStream_t s) {
  const uint32_t nc = batch_compact_chunks(b.n_blocks);
  if (nc == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bcount, dim3(nc), dim3(kCompactChunk), 0, s, b);
  hipLaunchKernelGGL(k_bscan, dim3(1), dim3(1024), 0, s, b, nc);
  hipLaunchKernelGGL(k_bwrite, dim3(nc), dim3(kCompactChunk), 0, s, b, nc);
  return hipGetLastError();
}

hipError_t launch_put_range(uint64_t* desc, uint64_t d_out, uint64_t lo, uint64_t hi, hipStream_t s) {
  hipLaunchKernelGGL(k_put_range, dim3(1), dim3(64), 0, s, desc, d_out, lo, hi);
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
