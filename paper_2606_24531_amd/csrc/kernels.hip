// gfx950 kernels of libaceseek: two-layer decode of absolute-offset LZ77
// archives (entropy layer: interleaved rANS; match layer: absolute-offset
// copies).  Paper Sections 2, 3 and 5; the rANS is Duda's, interleaved as in
// Giesen's construction (paper Section 9 cites both lines of work).
//
// Wave64 everywhere.  No MFMA: the path is integer decode and byte movement.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace ace {
namespace {

constexpr uint32_t kWave = 64;

__device__ __forceinline__ uint32_t ld16(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8);
}
__device__ __forceinline__ uint32_t ld32(const uint8_t* p) {
  return *reinterpret_cast<const uint32_t*>(p);  // callers pass 4-aligned addresses
}
__device__ __forceinline__ uint64_t ld64(const uint8_t* p) {
  return (uint64_t)ld32(p) | ((uint64_t)ld32(p + 4) << 32);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}


__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v, uint32_t lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(v, d, 64);
    if (lane >= (uint32_t)d) v += y;
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_total(uint32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ void flag(uint32_t* err, uint32_t bit) { atomicOr(err, bit); }

// ---------------------------------------------------------------------------
// Entropy layer: one wavefront decodes one rANS stream.
//
// LDS holds the stream's 12-bit table as a 4096-byte slot -> symbol map plus
// one packed word per symbol ((f-1) << 16 | cum), and a 4 KiB ring of
// renormalisation words refilled 1 KiB at a time from a register prefetch,
// so the decode loop never waits on HBM latency.  Lane j owns state j; each
// step decodes symbols t*W .. t*W+W-1, and the lanes that renormalise take
// consecutive words in lane order: word = running position +
// mbcnt(ballot(need)).  The loop body is branch-free apart from the
// wave-uniform ring refill.
// ---------------------------------------------------------------------------
struct RansSmem {
  uint8_t sym[4096];              // slot -> symbol
  uint4 ring[256];                // 4 chunks x 64 lanes x 16 B
  uint32_t fc[256];               // symbol -> (f-1) << 16 | cum
  uint8_t by_rank[256];           // k-th present symbol
  unsigned long long starts[64];  // bit t set: a symbol's interval starts at slot t
};

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Returns false (wave-uniform) when the stream breaks a format rule.
__device__ __forceinline__ bool rans_decode_wave(const uint8_t* src, uint32_t clen, uint32_t n, uint32_t W,
                                 uint8_t* dst, RansSmem& sm, uint32_t lane) {
  // ---- frequency table: 32-byte presence bitmap, then f-1 per present symbol
  if (clen < 32) return false;
  const uint32_t nib = ((uint32_t)src[lane >> 1] >> ((lane & 1) * 4)) & 0xFu;
  const uint32_t cnt = __popc(nib);
  const uint32_t before = wave_incl_sum(cnt, lane) - cnt;
  const uint32_t present = uniform(wave_total(cnt));
  const uint32_t tsz = (32 + 2 * present + 3) & ~3u;
  if (present == 0 || tsz + 4 * W > clen || ((clen - tsz - 4 * W) & 1)) return false;
  uint32_t f[4], mysum = 0, k = before;
#pragma unroll
  for (int j = 0; j < 4; j++) {
    f[j] = ((nib >> j) & 1) ? ld16(src + 32 + 2 * (k++)) + 1 : 0;
    mysum += f[j];
  }
  uint32_t cum = wave_incl_sum(mysum, lane) - mysum;
  if (uniform(wave_total(mysum)) != kM) return false;
  sm.starts[lane] = 0ull;
  wave_sync();
  k = before;
#pragma unroll
  for (int j = 0; j < 4; j++) {
    const uint32_t s = 4 * lane + j;
    sm.fc[s] = f[j] ? ((f[j] - 1) << 16) | cum : 0u;
    if (f[j]) {
      sm.by_rank[k++] = (uint8_t)s;
      atomicOr(&sm.starts[cum >> 6], 1ull << (cum & 63));
    }
    cum += f[j];
  }
  wave_sync();
  // ---- slot -> symbol: lane l fills slots 64l .. 64l+63 in order, the rank
  // of the covering symbol advancing at every interval start
  {
    const unsigned long long w = sm.starts[lane];
    const uint32_t pc = __popcll(w);
    int rank = (int)(wave_incl_sum(pc, lane) - pc) - 1;
    uint32_t* out32 = reinterpret_cast<uint32_t*>(sm.sym) + 16 * lane;
    uint32_t cur = rank >= 0 ? sm.by_rank[rank] : 0u;
    for (uint32_t q = 0; q < 16; q++) {
      uint32_t word = 0;
#pragma unroll
      for (uint32_t b = 0; b < 4; b++) {
        if ((w >> (4 * q + b)) & 1) cur = sm.by_rank[++rank];
        word |= cur << (8 * b);
      }
      out32[q] = word;
    }
  }
  // ---- states and word ring
  const uint8_t* wsrc = src + tsz + 4 * W;
  const uint32_t nwords = (clen - tsz - 4 * W) >> 1;
  uint32_t x = lane < W ? ld32(src + tsz + 4 * lane) : kL;
  if (__ballot(lane < W && x < kL)) return false;
  const uintptr_t a0 = (uintptr_t)wsrc & ~(uintptr_t)15;
  const uint32_t hw = uniform((uint32_t)((uintptr_t)wsrc - a0) >> 1);  // word 0 in chunk 0
  const uint32_t nchunks = uniform((2 * (hw + nwords) + 1023) >> 10);
  const uint4* gch = reinterpret_cast<const uint4*>(a0);
  uint32_t committed = 0;
  for (; committed < 3 && committed < nchunks; committed++)
    sm.ring[(committed & 3) * 64 + lane] = gch[committed * 64 + lane];
  uint4 pf = make_uint4(0, 0, 0, 0);
  if (committed < nchunks) pf = gch[committed * 64 + lane];
  wave_sync();
  const uint16_t* ring16 = reinterpret_cast<const uint16_t*>(sm.ring);
  uint32_t rp = hw;  // ring position (in words) of the next unread word
  const bool lane_on = lane < W;
  const uint32_t nsteps = uniform((n + W - 1) / W);
  uint32_t i = lane;
  for (uint32_t t = 0; t < nsteps; t++) {
    if (rp + 64 > committed * 512 && committed < nchunks) {  // wave-uniform
      sm.ring[(committed & 3) * 64 + lane] = pf;
      committed++;
      if (committed < nchunks) pf = gch[committed * 64 + lane];
      wave_sync();
    }
    const bool act = lane_on && i < n;
    const uint32_t slot = x & (kM - 1);
    const uint32_t s = sm.sym[slot];
    const uint32_t e = sm.fc[s];
    const uint32_t xs = x >> kProbBits;
    const uint32_t xn = __umul24(e >> 16, xs) + xs + slot - (e & 0xFFFu);
    const bool need = act && xn < kL;
    const uint64_t m = __ballot(need);
    const uint32_t pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, rp));
    uint32_t wd = ring16[pos & 2047];
    __asm__ volatile("" : "+v"(wd));  // read for every lane: keeps the update branch-free
    const uint32_t xa = act ? xn : x;
    x = need ? ((xn << 16) | wd) : xa;
    rp += (uint32_t)__popcll(m);
    if (act) dst[i] = (uint8_t)s;
    i += W;
  }
  const bool bad = rp - hw != nwords || (lane_on && x != kL);
  return __ballot(bad) == 0;
}

// Kernel (a): grid (n_plan, 3), one wavefront per (block, stream).  Decodes
// LIT into lit + plan_index * B, LEN into lens + 4 * seq_base and OFF into
// offs + ow * seq_base, and records where the block's bytes will live.
__global__ __launch_bounds__(64) void k_rans(DecodeArgs a) {
  __shared__ RansSmem sm;
  const uint32_t i = blockIdx.x, t = blockIdx.y, lane = threadIdx.x;
  if (a.n_plan_dev && i >= *a.n_plan_dev) return;
  const PlanEntry pe = a.plan[i];
  const uint8_t* be = a.arch + kHdr + (uint64_t)kBlk * pe.block;
  const uint64_t pay = ld64(be);
  if (t == 0 && lane == 0) a.loc[pe.block] = a.dst_base + pe.dst;
  const uint8_t* d = a.arch + pay + kSDesc * t;
  const uint32_t mode = d[0], n = ld32(d + 4), clen = ld32(d + 8), off = ld32(d + 12);
  uint8_t* dst = t == 0 ? a.lit + (uint64_t)i * a.B
               : t == 1 ? a.lens + 4ull * pe.seq_base
                        : a.offs + (uint64_t)a.ow * pe.seq_base;
  const uint8_t* src = a.arch + pay + off;
  if (mode == 0) return;  // raw streams are read in place by the expansion
  if (!rans_decode_wave(src, clen, n, a.W, dst, sm, lane) && lane == 0) flag(a.err, kErrCorrupt);
}

// ---------------------------------------------------------------------------
// Match layer: expansion of one block by a workgroup of kTile threads.
//
// Sequences are taken kTile at a time (one per thread).  A workgroup scan of
// L_k + M_k and L_k gives every sequence its block-relative start and its
// first literal, and each thread classifies its sequence's source once: a
// match byte i of sequence k reads absolute position O_k + (i mod d_k), with
// d_k = (match start) - O_k, so overlapping matches repeat with that period
// and every source lies before the match.  When all of a match's source
// bytes sit in one earlier block (found through the location table) or in an
// earlier tile of this block, a single base address serves every byte.
// Then every thread produces 16 contiguous output bytes at a time: one binary
// search for the first byte's sequence, then a forward walk; literal and
// match bytes each cost one address and one byte load, and a whole aligned
// chunk is written as one 16-byte store.  Sources that span blocks, or lie
// inside the tile being produced, take the slow path: follow the source back
// (to a literal, an earlier tile or an earlier block) -- each step moves
// strictly backwards, so the walk ends.
// ---------------------------------------------------------------------------
constexpr uint32_t kPoison = 1u, kSlow = 2u;

template <uint32_t kTile>
struct ExpandSmem {
  static constexpr uint32_t kRound = 4 * kTile;  // chunks sorted per round
  uint32_t list[kRound]; // chunk << 8 | sequence: copy chunks first, per-byte chunks from the back
  uint32_t nvec, nbyte;
  uint32_t dst[kTile];   // block-relative start of the sequence
  uint32_t lm[kTile];    // L | M << 16
  uint32_t dist[kTile];  // match start - O
  uint32_t flags[kTile]; // kPoison, kSlow
  uint64_t O[kTile];
  uint64_t lit[kTile];   // address of the sequence's first literal
  uint64_t mbase[kTile]; // address of absolute position 0 for this match's source
  uint32_t scan[8];
};

// Inclusive scans of a and b over the workgroup (kTile threads) and totals.
template <uint32_t kTile>
__device__ __forceinline__ void wg_scan2(uint32_t a, uint32_t b, uint32_t& ia, uint32_t& ib,
                                         uint32_t& ta, uint32_t& tb, uint32_t* sh) {
  constexpr uint32_t kW = kTile / 64;
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  a = wave_incl_sum(a, lane);
  b = wave_incl_sum(b, lane);
  if (kW == 1) {
    ta = __shfl(a, 63, 64);
    tb = __shfl(b, 63, 64);
    ia = a;
    ib = b;
    return;
  }
  __syncthreads();
  if (lane == 63) {
    sh[w] = a;
    sh[4 + w] = b;
  }
  __syncthreads();
  uint32_t oa = 0, ob = 0;
  for (uint32_t j = 0; j < w; j++) {
    oa += sh[j];
    ob += sh[4 + j];
  }
  ta = tb = 0;
  for (uint32_t j = 0; j < kW; j++) {
    ta += sh[j];
    tb += sh[4 + j];
  }
  ia = a + oa;
  ib = b + ob;
}

__device__ __forceinline__ uint32_t find_seq(const uint32_t* sdst, uint32_t cnt, uint32_t p) {
  uint32_t lo = 0, hi = cnt;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (sdst[mid] <= p) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ bool dep_listed(const uint32_t* deps, uint32_t cnt, uint32_t c) {
  uint32_t lo = 0, hi = cnt;
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    uint32_t v = deps[mid];
    if (v == c) return true;
    if (v < c) lo = mid + 1; else hi = mid;
  }
  return false;
}

struct BlockCtx {
  uint64_t bs;       // absolute start of the block
  uint32_t blen, n_lit, d0, cnt;
  uint8_t* out;      // the block's first byte
  bool ext_ok;
};

// Slow path: the byte at block-relative p, following sources back.
template <uint32_t kTile>
__device__ uint8_t resolve_slow(const DecodeArgs& a, const ExpandSmem<kTile>& sm, const BlockCtx& c,
                                uint32_t p, uint32_t& n_ext) {
  for (;;) {
    const uint32_t s = find_seq(sm.dst, c.cnt, p);
    if (sm.flags[s] & kPoison) return 0;
    const uint32_t r = p - sm.dst[s];
    const uint32_t Ls = sm.lm[s] & 0xFFFFu;
    if (r < Ls) return *reinterpret_cast<const uint8_t*>(sm.lit[s] + r);
    const uint32_t ii = r - Ls, d = sm.dist[s];
    const uint64_t src = sm.O[s] + (ii < d ? ii : ii % d);
    if (src < c.bs) {
      if (!c.ext_ok) return 0;  // a dependency never published: read nothing
      const uint64_t blk = src / a.B;
      n_ext++;
      return reinterpret_cast<const uint8_t*>(a.loc[blk])[src - blk * a.B];
    }
    const uint32_t q = (uint32_t)(src - c.bs);
    if (q < c.d0) return c.out[q];
    p = q;
  }
}

// Expands plan entry i.  Sources in earlier blocks must be complete and
// visible (unless ext_ok is false, after a timed-out wait).
template <uint32_t kTile>
__device__ __forceinline__ void expand_block(const DecodeArgs& a, uint32_t i, ExpandSmem<kTile>& sm,
                                             bool ext_ok = true) {
  const uint32_t tid = threadIdx.x;
  const PlanEntry pe = a.plan[i];
  const uint32_t b = pe.block;
  const uint8_t* be = a.arch + kHdr + (uint64_t)kBlk * b;
  const uint64_t pay = ld64(be);
  const uint32_t n_seq = ld32(be + 12), dep_off = ld32(be + 20), dep_cnt = ld32(be + 24);
  const uint32_t* deps = reinterpret_cast<const uint32_t*>(a.arch + kHdr + (uint64_t)kBlk * a.n_blocks) + dep_off;
  BlockCtx c;
  c.n_lit = ld32(a.arch + pay + 4);
  c.bs = (uint64_t)b * a.B;
  c.blen = (uint32_t)((a.n_total - c.bs) < a.B ? (a.n_total - c.bs) : a.B);
  c.out = reinterpret_cast<uint8_t*>(a.dst_base + pe.dst);
  c.ext_ok = ext_ok;
  // each stream is read in place when stored raw, else from its decoded copy
  const uint8_t* pl = a.arch + pay;
  const uint8_t* lit = pl[0] == 0 ? pl + ld32(pl + 12) : a.lit + (uint64_t)i * a.B;
  const uint8_t* lens = pl[16] == 0 ? pl + ld32(pl + 28) : a.lens + 4ull * pe.seq_base;
  const uint8_t* offs = pl[32] == 0 ? pl + ld32(pl + 44) : a.offs + (uint64_t)a.ow * pe.seq_base;
  const bool aligned = (((uintptr_t)c.out) & 15) == 0;
  constexpr uint32_t kRound = ExpandSmem<kTile>::kRound;
  uint32_t carry_pos = 0, carry_lit = 0, n_ext = 0;
  bool bad = false;
  for (uint32_t t0 = 0; t0 < n_seq; t0 += kTile) {
    const uint32_t k = t0 + tid;
    const bool valid = k < n_seq;
    uint32_t L = 0, M = 0;
    uint64_t O = 0;
    if (valid) {
      const uint32_t lm = ld32(lens + 4ull * k);
      L = lm & 0xFFFFu;
      M = lm >> 16;
      O = a.ow == 4 ? (uint64_t)ld32(offs + 4ull * k) : ld64(offs + 8ull * k);
    }
    uint32_t ip, il, tp, tl;
    wg_scan2<kTile>(L + M, L, ip, il, tp, tl, sm.scan);
    const uint32_t dst = carry_pos + ip - (L + M);
    const uint32_t litk = carry_lit + il - L;
    const uint32_t d0 = carry_pos;
    uint32_t fl = 0, dist = 0;
    uint64_t mbase = 0;
    if (valid) {
      const uint64_t mabs = c.bs + dst + L;
      if ((uint64_t)dst + L + M > c.blen || (uint64_t)litk + L > c.n_lit) fl = kPoison;
      if (M && !fl) {
        if (O >= mabs) {
          fl = kPoison;
        } else {
          dist = (uint32_t)((mabs - O) < 0xFFFFFFFFull ? (mabs - O) : 0xFFFFFFFFull);
          const uint64_t src_hi = O + (M < dist ? M : dist);  // bytes actually read
          if (O < c.bs) {
            // every earlier block the source touches must be a listed dependency
            const uint64_t end = src_hi < c.bs ? src_hi : c.bs;
            for (uint64_t blk = O / a.B; blk * a.B < end; blk++)
              if (!dep_listed(deps, dep_cnt, (uint32_t)blk)) {
                fl = kPoison;
                break;
              }
          }
          if (!fl) {
            const uint64_t b0 = O / a.B, b1 = (src_hi - 1) / a.B;
            if (src_hi <= c.bs && b0 == b1 && ext_ok) {
              mbase = a.loc[b0] - b0 * a.B;  // one earlier block
              n_ext += M;
            } else if (O >= c.bs && src_hi - c.bs <= d0) {
              mbase = (uint64_t)(uintptr_t)c.out - c.bs;  // an earlier tile of this block
            } else {
              fl = kSlow;
            }
          }
        }
      } else if (!M && O != 0) {
        bad = true;
      }
      if (fl & kPoison) bad = true;
    }
    sm.dst[tid] = dst;
    sm.lm[tid] = L | (M << 16);
    sm.dist[tid] = dist;
    sm.flags[tid] = fl;
    sm.O[tid] = O;
    sm.lit[tid] = (uint64_t)(uintptr_t)lit + litk;
    sm.mbase[tid] = mbase;
    __syncthreads();
    c.d0 = d0;
    c.cnt = (n_seq - t0) < kTile ? (n_seq - t0) : kTile;
    const uint64_t d1w = (uint64_t)carry_pos + tp;
    const uint32_t d1 = d1w < c.blen ? (uint32_t)d1w : c.blen;
    // Output is produced in 16-byte chunks, 4 per thread per round.  Each
    // round first sorts its chunks: a chunk whose 16 bytes come from one
    // contiguous source (all literals of one sequence, or one match with no
    // period wrap) is copied with five aligned dword loads and one 16-byte
    // store; the others go through the per-byte path.  Sorting keeps the two
    // kinds of work in separate passes, so a wavefront does not pay for both.
    const uint32_t base = d0 & ~15u;
    const uint32_t nch = d1 > base ? (d1 - base + 15) / 16 : 0;
    const bool pow2 = (a.B & (a.B - 1)) == 0;
    for (uint32_t k0 = 0; k0 < nch; k0 += kRound) {
      const uint32_t kn = nch - k0 < kRound ? nch - k0 : kRound;
      if (tid == 0) {
        sm.nvec = 0;
        sm.nbyte = 0;
      }
      __syncthreads();
      for (uint32_t k = k0 + tid; k < k0 + kn; k += kTile) {
        const uint32_t cb = base + 16 * k;
        const uint32_t p0 = cb < d0 ? d0 : cb;
        const uint32_t pe1 = cb + 16 < d1 ? cb + 16 : d1;
        const uint32_t sq = find_seq(sm.dst, c.cnt, p0);
        bool vec = aligned && p0 == cb && pe1 == cb + 16 && !(sm.flags[sq] & kPoison);
        if (vec) {
          const uint32_t end_s = sq + 1 < c.cnt ? sm.dst[sq + 1] : d1;
          const uint32_t r0 = cb - sm.dst[sq], Ls = sm.lm[sq] & 0xFFFFu;
          if (cb + 16 > end_s) {
            vec = false;
          } else if (r0 + 16 <= Ls) {
            vec = true;  // all literals (the literal scratch has readable slack)
          } else if (r0 >= Ls && sm.flags[sq] == 0 && pow2) {
            // the five aligned dwords must stay inside the source block's bytes
            const uint32_t ii0 = r0 - Ls;
            const uint64_t src = sm.O[sq] + ii0;
            const uint32_t off = (uint32_t)(src & (a.B - 1));
            const uint32_t shp = (uint32_t)((sm.mbase[sq] + src) & 3);
            const uint32_t limit = src >= c.bs ? c.blen : a.B;
            vec = ii0 + 16 <= sm.dist[sq] && off >= shp && off - shp + 20 <= limit;
          } else {
            vec = false;
          }
        }
        const uint32_t e = (k << 8) | sq;
        if (vec) sm.list[atomicAdd(&sm.nvec, 1u)] = e;
        else sm.list[kRound - 1 - atomicAdd(&sm.nbyte, 1u)] = e;
      }
      __syncthreads();
      const uint32_t nv = sm.nvec, nby = sm.nbyte;
      for (uint32_t ei = tid; ei < nv; ei += kTile) {
        const uint32_t e = sm.list[ei], k = e >> 8, sq = e & 0xFFu;
        const uint32_t cb = base + 16 * k;
        const uint32_t r0 = cb - sm.dst[sq], Ls = sm.lm[sq] & 0xFFFFu;
        const uint8_t* src = r0 < Ls ? reinterpret_cast<const uint8_t*>(sm.lit[sq] + r0)
                                     : reinterpret_cast<const uint8_t*>(sm.mbase[sq] + sm.O[sq] + (r0 - Ls));
        const uint32_t sh = (uint32_t)((uintptr_t)src & 3);
        const uint32_t* w = reinterpret_cast<const uint32_t*>(src - sh);
        const uint32_t w0 = w[0], w1 = w[1], w2 = w[2], w3 = w[3], w4 = w[4];
        *reinterpret_cast<uint4*>(c.out + cb) =
            make_uint4(__builtin_amdgcn_alignbyte(w1, w0, sh), __builtin_amdgcn_alignbyte(w2, w1, sh),
                       __builtin_amdgcn_alignbyte(w3, w2, sh), __builtin_amdgcn_alignbyte(w4, w3, sh));
      }
      for (uint32_t ei = tid; ei < nby; ei += kTile) {
        const uint32_t e = sm.list[kRound - 1 - ei], k = e >> 8;
        const uint32_t cb = base + 16 * k;
        const uint32_t p0 = cb < d0 ? d0 : cb;
        const uint32_t pe1 = cb + 16 < d1 ? cb + 16 : d1;
        uint32_t s = e & 0xFFu;
        uint32_t s_end = s + 1 < c.cnt ? sm.dst[s + 1] : d1;
        uint32_t acc[4] = {0, 0, 0, 0};
#pragma unroll
        for (uint32_t j = 0; j < 16; j++) {
          const uint32_t p = cb + j;
          uint32_t v = 0;
          if (p >= p0 && p < pe1) {
            while (p >= s_end) {
              s++;
              s_end = s + 1 < c.cnt ? sm.dst[s + 1] : d1;
            }
            const uint32_t r = p - sm.dst[s];
            const uint32_t Ls = sm.lm[s] & 0xFFFFu;
            const uint32_t f = sm.flags[s];
            if (f & kPoison) {
              v = 0;  // a format rule failed: write zeros, read nothing
            } else if (r < Ls) {
              v = *reinterpret_cast<const uint8_t*>(sm.lit[s] + r);
            } else if (f == 0) {
              const uint32_t ii = r - Ls, d = sm.dist[s];
              v = *reinterpret_cast<const uint8_t*>(sm.mbase[s] + sm.O[s] + (ii < d ? ii : ii % d));
            } else {
              v = resolve_slow<kTile>(a, sm, c, p, n_ext);
            }
          }
          acc[j >> 2] |= v << (8 * (j & 3));
        }
        if (aligned && p0 == cb && pe1 == cb + 16) {
          *reinterpret_cast<uint4*>(c.out + cb) = make_uint4(acc[0], acc[1], acc[2], acc[3]);
        } else {
#pragma unroll
          for (uint32_t j = 0; j < 16; j++)
            if (cb + j >= p0 && cb + j < pe1) c.out[cb + j] = (uint8_t)(acc[j >> 2] >> (8 * (j & 3)));
        }
      }
      __syncthreads();
    }
    carry_pos = (uint32_t)(d1w > 0xFFFFFFFFull ? 0xFFFFFFFFu : d1w);
    carry_lit += tl;
    __syncthreads();
    if ((uint64_t)carry_pos > c.blen) {
      bad = true;
      break;
    }
  }
  if (tid == 0 && (carry_pos != c.blen || carry_lit > c.n_lit)) bad = true;
  if (bad) flag(a.err, kErrCorrupt);
  n_ext = wave_total(n_ext);
  if ((tid & 63) == 0 && n_ext) atomicAdd(a.ext_bytes, (unsigned long long)n_ext);
}

// level < 0: plan entries plan_lo + blockIdx.x; else the level's plan range
// is read from device memory.
__global__ __launch_bounds__(256) void k_expand(DecodeArgs a, uint32_t plan_lo, int level) {
  __shared__ ExpandSmem<256> sm;
  uint32_t i = plan_lo + blockIdx.x;
  if (level >= 0) {
    i = a.lvl_dev[level] + blockIdx.x;
    if (i >= a.lvl_dev[level + 1]) return;
  }
  expand_block<256>(a, i, sm);
}

// ---------------------------------------------------------------------------
// Kernel (c): persistent, dependency-ordered decode.  Each single-wave
// workgroup repeatedly takes the next plan entry (the plan lists blocks by
// increasing dependency level), entropy-decodes its three streams, waits
// until every block its matches read from has published completion, expands
// it, and publishes its own completion.  A wave only ever waits for blocks
// taken earlier, and those are held by running waves, so the wait always
// ends; it is bounded anyway and flags a timeout instead of hanging.
// Cross-XCD visibility: completion is a release store at agent scope (it
// writes back this XCD's L2), the wait an acquire load at agent scope.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void decode_stream(const DecodeArgs& a, const PlanEntry& pe, uint32_t i,
                                              uint32_t t, RansSmem& sm, uint32_t lane) {
  const uint8_t* be = a.arch + kHdr + (uint64_t)kBlk * pe.block;
  const uint64_t pay = ld64(be);
  const uint8_t* d = a.arch + pay + kSDesc * t;
  const uint32_t mode = d[0], n = ld32(d + 4), clen = ld32(d + 8), off = ld32(d + 12);
  uint8_t* dst = t == 0 ? a.lit + (uint64_t)i * a.B
               : t == 1 ? a.lens + 4ull * pe.seq_base
                        : a.offs + (uint64_t)a.ow * pe.seq_base;
  const uint8_t* src = a.arch + pay + off;
  if (mode == 0) {
    for (uint32_t j = lane; j < n; j += kWave) dst[j] = src[j];
  } else if (!rans_decode_wave(src, clen, n, a.W, dst, sm, lane) && lane == 0) {
    flag(a.err, kErrCorrupt);
  }
}

__global__ __launch_bounds__(64) void k_persist(DecodeArgs a) {
  __shared__ RansSmem rs;
  __shared__ ExpandSmem<64> es;
  const uint32_t lane = threadIdx.x;
  const uint32_t n_plan = a.n_plan_dev ? *a.n_plan_dev : a.n_plan;
  for (;;) {
    uint32_t i = 0;
    if (lane == 0) i = atomicAdd(a.queue, 1u);
    i = __shfl(i, 0, 64);
    if (i >= n_plan) break;
    const PlanEntry pe = a.plan[i];
    if (lane == 0) a.loc[pe.block] = a.dst_base + pe.dst;
    decode_stream(a, pe, i, 1, rs, lane);
    decode_stream(a, pe, i, 2, rs, lane);
    decode_stream(a, pe, i, 0, rs, lane);
    // dependencies: every listed earlier block must have published
    const uint8_t* be = a.arch + kHdr + (uint64_t)kBlk * pe.block;
    const uint32_t dep_off = ld32(be + 20), dep_cnt = ld32(be + 24);
    const uint32_t* deps = reinterpret_cast<const uint32_t*>(a.arch + kHdr + (uint64_t)kBlk * a.n_blocks) + dep_off;
    // Poll with relaxed loads (no cache invalidation per poll), then acquire
    // once.  The wait is bounded in time (the 100 MHz constant clock), and
    // once any wave has given up every other wait gives up at once, so the
    // kernel always drains.
    bool timeout = false;
    const uint64_t t_start = wall_clock64();
    for (uint32_t j = lane; j < dep_cnt; j += kWave) {
      const uint32_t* f = a.done + deps[j];
      while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != a.epoch) {
        if (wall_clock64() - t_start > a.wait_ticks ||
            (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrTimeout)) {
          timeout = true;
          break;
        }
        __builtin_amdgcn_s_sleep(8);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const bool late = __ballot(timeout) != 0;
    if (late && lane == 0) flag(a.err, kErrTimeout);
    __syncthreads();  // streams of this block written, dependencies visible to all lanes
    expand_block<64>(a, i, es, !late);
    __syncthreads();
    if (lane == 0) __hip_atomic_store(a.done + pe.block, a.epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------
// Copy of decoded ranges (seek clipping and batched gathers): one workgroup
// per item, 16 contiguous bytes per thread per pass, source blocks found via
// the location table.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_copy(DecodeArgs a, const CopyItem* items) {
  const CopyItem it = items[blockIdx.x];
  uint8_t* dst = reinterpret_cast<uint8_t*>(it.dst);
  for (uint32_t j0 = threadIdx.x * 16; j0 < it.len; j0 += 256 * 16) {
    uint64_t pos = it.src_abs + j0;
    uint64_t c = pos / a.B;
    uint64_t cend = (c + 1) * a.B;
    const uint8_t* base = reinterpret_cast<const uint8_t*>(a.loc[c]) - c * a.B;
    uint32_t jn = j0 + 16 < it.len ? j0 + 16 : it.len;
    for (uint32_t j = j0; j < jn; j++, pos++) {
      if (pos >= cend) {
        c++;
        cend += a.B;
        base = reinterpret_cast<const uint8_t*>(a.loc[c]) - c * a.B;
      }
      dst[j] = base[pos];
    }
  }
}

// ---------------------------------------------------------------------------
// Device-side planning of a seek batch.  Mark the target blocks of every
// request; close the set under the dependency lists level by level from the
// top (dependencies always sit at lower levels); compact the marked blocks,
// in level order, into a plan whose entries decode into workspace slots;
// after the decode, gather each request's range to its output offset.
// ---------------------------------------------------------------------------
__global__ void k_bmark(BatchArgs b) {
  const uint64_t n = b.desc[0];
  for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < n;
       r += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t lo = b.desc[2 + 3 * r], hi = b.desc[3 + 3 * r];
    if (hi <= lo || hi > b.n_total) continue;
    for (uint64_t blk = lo / b.B; blk <= (hi - 1) / b.B; blk++) b.need[blk] = 1;
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
    for (uint32_t k = 0; k < dep_cnt; k++) b.need[deps[k]] = 1;
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
    if (f) b.plan[pos] = PlanEntry{blk, seq, (uint64_t)pos * b.B};
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
  const uint64_t len = hi - lo;
  for (uint64_t j0 = threadIdx.x * 16ull; j0 < len; j0 += 256 * 16) {
    uint64_t pos = lo + j0;
    uint64_t c = pos / a.B;
    uint64_t cend = (c + 1) * a.B;
    const uint8_t* base = reinterpret_cast<const uint8_t*>(b.loc[c]) - c * a.B;
    const uint64_t jn = j0 + 16 < len ? j0 + 16 : len;
    for (uint64_t j = j0; j < jn; j++, pos++) {
      if (pos >= cend) {
        c++;
        cend += a.B;
        base = reinterpret_cast<const uint8_t*>(b.loc[c]) - c * a.B;
      }
      dst[j] = base[pos];
    }
  }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint64_t n) {
  for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < n;
       j += (uint64_t)gridDim.x * blockDim.x)
    p[j] = v;
}

}  // namespace

hipError_t launch_rans(const DecodeArgs& a, hipStream_t s) {
  if (a.n_plan == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rans, dim3(a.n_plan, 3), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_expand_level(const DecodeArgs& a, uint32_t lo, uint32_t hi, hipStream_t s) {
  if (hi <= lo) return hipSuccess;
  hipLaunchKernelGGL(k_expand, dim3(hi - lo), dim3(256), 0, s, a, lo, -1);
  return hipGetLastError();
}

hipError_t launch_rans_dev(const DecodeArgs& a, uint32_t grid, hipStream_t s) {
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rans, dim3(grid, 3), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_expand_level_dev(const DecodeArgs& a, uint32_t level, uint32_t width,
                                   hipStream_t s) {
  if (width == 0) return hipSuccess;
  hipLaunchKernelGGL(k_expand, dim3(width), dim3(256), 0, s, a, 0u, (int)level);
  return hipGetLastError();
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
    static int cached = 0;
    if (cached == 0) {
      int dev = 0, cus = 0, per_cu = 0;
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
          hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persist, 64, 0) != hipSuccess)
        return hipErrorUnknown;
      cached = cus * (per_cu > 0 ? per_cu : 1);
    }
    grid = (uint32_t)cached;
  }
  if (grid > a.n_plan) grid = a.n_plan;
  hipLaunchKernelGGL(k_persist, dim3(grid), dim3(64), 0, s, a);
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

}  // namespace ace
