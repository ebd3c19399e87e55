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

__device__ __forceinline__ uint32_t mbcnt64(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
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
// LDS: a 4096-entry slot table (entry = symbol | (f-1) << 8 | (slot-cum) << 20)
// and a 4 KiB ring of renormalisation words refilled 1 KiB at a time from a
// register prefetch, so the decode loop never waits on HBM latency.  Lane j
// owns state j; each step decodes symbols t*W .. t*W+W-1, and the lanes that
// renormalise take consecutive words in lane order: word index = running base
// + mbcnt(ballot(need)).
// ---------------------------------------------------------------------------
struct RansSmem {
  uint32_t lut[4096];
  uint4 ring[256];            // 4 chunks x 64 lanes x 16 B
  uint32_t pk[256];           // per present symbol (by rank): s | (f-1)<<8 | cum<<20
  unsigned long long starts[64];  // bit t set: a symbol's interval starts at slot t
};

// Returns false (wave-uniform) when the stream breaks a format rule.
__device__ bool rans_decode_wave(const uint8_t* src, uint32_t clen, uint32_t n, uint32_t W,
                                 uint8_t* dst, RansSmem& sm, uint32_t lane) {
  // ---- frequency table: 32-byte presence bitmap, then f-1 per present symbol
  if (clen < 32) return false;
  uint32_t nib = ((uint32_t)src[lane >> 1] >> ((lane & 1) * 4)) & 0xFu;
  uint32_t cnt = __popc(nib);
  uint32_t before = wave_incl_sum(cnt, lane) - cnt;
  uint32_t present = wave_total(cnt);
  uint32_t tsz = (32 + 2 * present + 3) & ~3u;
  if (present == 0 || tsz + 4 * W > clen || ((clen - tsz - 4 * W) & 1)) return false;
  uint32_t f[4], mysum = 0, k = before;
#pragma unroll
  for (int j = 0; j < 4; j++) {
    f[j] = ((nib >> j) & 1) ? ld16(src + 32 + 2 * (k++)) + 1 : 0;
    mysum += f[j];
  }
  uint32_t cum = wave_incl_sum(mysum, lane) - mysum;
  if (wave_total(mysum) != kM) return false;
  sm.starts[lane] = 0ull;
  wave_sync();
  k = before;
#pragma unroll
  for (int j = 0; j < 4; j++) {
    if (f[j]) {
      sm.pk[k++] = (4 * lane + j) | ((f[j] - 1) << 8) | (cum << 20);
      atomicOr(&sm.starts[cum >> 6], 1ull << (cum & 63));
    }
    cum += f[j];
  }
  wave_sync();
  // ---- slot table: lane l fills slots 64l .. 64l+63.  The symbol of slot t
  // is the one of rank (starts at or before t) - 1; the visiting order is
  // rotated per lane so that the 64 lanes write 64 different banks.
  {
    unsigned long long w = sm.starts[lane];
    uint32_t pc = __popcll(w);
    uint32_t rank0 = wave_incl_sum(pc, lane) - pc;
    for (uint32_t t = 0; t < 64; t++) {
      uint32_t tt = t ^ lane;
      uint32_t rank = rank0 + __popcll(w & (~0ull >> (63 - tt))) - 1;
      uint32_t e = sm.pk[rank];
      uint32_t slot = 64 * lane + tt;
      sm.lut[slot] = (e & 0xFFFFFu) | ((slot - (e >> 20)) << 20);
    }
  }
  // ---- states and word ring
  const uint8_t* wsrc = src + tsz + 4 * W;
  uint32_t nwords = (clen - tsz - 4 * W) >> 1;
  uint32_t x = lane < W ? ld32(src + tsz + 4 * lane) : kL;
  if (__ballot(lane < W && x < kL)) return false;
  const uintptr_t a0 = (uintptr_t)wsrc & ~(uintptr_t)15;
  const uint32_t hw = (uint32_t)((uintptr_t)wsrc - a0) >> 1;  // word 0's position in chunk 0
  const uint32_t nchunks = (2 * (hw + nwords) + 1023) >> 10;
  const uint4* gch = reinterpret_cast<const uint4*>(a0);
  uint32_t committed = 0;
  for (; committed < 3 && committed < nchunks; committed++)
    sm.ring[(committed & 3) * 64 + lane] = gch[committed * 64 + lane];
  uint4 pf = make_uint4(0, 0, 0, 0);
  if (committed < nchunks) pf = gch[committed * 64 + lane];
  wave_sync();
  const uint16_t* ring16 = reinterpret_cast<const uint16_t*>(sm.ring);
  uint32_t wpos = 0;
  bool over = false;
  const uint32_t nsteps = (n + W - 1) / W;
  for (uint32_t t = 0; t < nsteps; t++) {
    if (2 * (hw + wpos + 64) > committed * 1024 && committed < nchunks) {
      sm.ring[(committed & 3) * 64 + lane] = pf;
      committed++;
      if (committed < nchunks) pf = gch[committed * 64 + lane];
      wave_sync();
    }
    uint32_t i = t * W + lane;
    bool act = lane < W && i < n;
    uint32_t e = sm.lut[x & (kM - 1)];
    uint32_t xn = (((e >> 8) & 0xFFFu) + 1) * (x >> kProbBits) + (e >> 20);
    bool need = act && xn < kL;
    uint64_t m = __ballot(need);
    if (need) {
      uint32_t kk = wpos + mbcnt64(m);
      over |= kk >= nwords;
      x = (xn << 16) | ring16[(hw + kk) & 2047];
    } else if (act) {
      x = xn;
    }
    wpos += __popcll(m);
    if (act) dst[i] = (uint8_t)e;
  }
  bool bad = over || wpos != nwords || (lane < W && x != kL);
  return __ballot(bad) == 0;
}

// Kernel (a): grid (n_plan, 3), one wavefront per (block, stream).  Decodes
// LIT into lit + plan_index * B, LEN into lens + 4 * seq_base and OFF into
// offs + ow * seq_base, and records where the block's bytes will live.
__global__ __launch_bounds__(64) void k_rans(DecodeArgs a) {
  __shared__ RansSmem sm;
  const uint32_t i = blockIdx.x, t = blockIdx.y, lane = threadIdx.x;
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
  if (mode == 0) {
    for (uint32_t j = lane; j < n; j += kWave) dst[j] = src[j];
    return;
  }
  if (!rans_decode_wave(src, clen, n, a.W, dst, sm, lane) && lane == 0) flag(a.err, kErrCorrupt);
}

// ---------------------------------------------------------------------------
// Match layer: expansion of one block by a 256-thread workgroup.
//
// Sequences are taken 256 at a time (one per thread); a workgroup scan of
// L_k + M_k and L_k gives every sequence its block-relative start and its
// first literal.  Then every output byte of the tile is produced by its own
// thread: the sequence holding it is found by binary search; a literal is
// read from the decoded LIT stream; a match byte i of sequence k reads
// absolute position O_k + (i mod (dst_k - O_k)) (overlapping matches repeat
// with that period), which lies before the match.  A source in an earlier
// block is read through the location table; one in an earlier tile of this
// block is already written; one inside this tile is followed further (to a
// literal, an earlier tile or an earlier block) -- each step moves strictly
// backwards, so the walk ends.
// ---------------------------------------------------------------------------
constexpr uint32_t kPoison = 0x80000000u;

template <uint32_t kTile>
struct ExpandSmem {
  uint32_t dst[kTile];  // block-relative start of the sequence
  uint32_t L[kTile];
  uint32_t M[kTile];    // bit 31: poisoned (a format rule failed)
  uint32_t lit[kTile];  // index of the first literal
  uint64_t O[kTile];
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

// Expands plan entry i with kTile threads.  Sources in earlier blocks must be
// complete and visible.
template <uint32_t kTile>
__device__ void expand_block(const DecodeArgs& a, uint32_t i, ExpandSmem<kTile>& sm) {
  const uint32_t tid = threadIdx.x;
  const PlanEntry pe = a.plan[i];
  const uint32_t b = pe.block;
  const uint8_t* be = a.arch + kHdr + (uint64_t)kBlk * b;
  const uint64_t pay = ld64(be);
  const uint32_t n_seq = ld32(be + 12), dep_off = ld32(be + 20), dep_cnt = ld32(be + 24);
  const uint32_t* deps = reinterpret_cast<const uint32_t*>(a.arch + kHdr + (uint64_t)kBlk * a.n_blocks) + dep_off;
  const uint32_t n_lit = ld32(a.arch + pay + 4);
  const uint64_t bs = (uint64_t)b * a.B;
  const uint32_t blen = (uint32_t)((a.n_total - bs) < a.B ? (a.n_total - bs) : a.B);
  uint8_t* out = reinterpret_cast<uint8_t*>(a.dst_base + pe.dst);
  const uint8_t* lit = a.lit + (uint64_t)i * a.B;
  const uint8_t* lens = a.lens + 4ull * pe.seq_base;
  const uint8_t* offs = a.offs + (uint64_t)a.ow * pe.seq_base;
  uint32_t carry_pos = 0, carry_lit = 0, n_ext = 0;
  bool bad = false;
  for (uint32_t t0 = 0; t0 < n_seq; t0 += kTile) {
    const uint32_t k = t0 + tid;
    const bool valid = k < n_seq;
    uint32_t L = 0, M = 0;
    uint64_t O = 0;
    if (valid) {
      uint32_t lm = ld32(lens + 4ull * k);
      L = lm & 0xFFFFu;
      M = lm >> 16;
      O = a.ow == 4 ? (uint64_t)ld32(offs + 4ull * k) : ld64(offs + 8ull * k);
    }
    uint32_t ip, il, tp, tl;
    wg_scan2<kTile>(L + M, L, ip, il, tp, tl, sm.scan);
    const uint32_t dst = carry_pos + ip - (L + M);
    const uint32_t litk = carry_lit + il - L;
    uint32_t mflag = M;
    if (valid) {
      const uint64_t mabs = bs + dst + L;
      bool poison = (uint64_t)dst + L + M > blen || (uint64_t)litk + L > n_lit;
      if (M) {
        if (O >= mabs) {
          poison = true;
        } else if (O < bs) {
          // every earlier block the source touches must be a listed dependency
          uint64_t end = O + M < bs ? O + M : bs;
          for (uint64_t c = O / a.B; c * a.B < end; c++)
            if (!dep_listed(deps, dep_cnt, (uint32_t)c)) {
              poison = true;
              break;
            }
        }
      } else if (O != 0) {
        bad = true;
      }
      if (poison) {
        bad = true;
        mflag |= kPoison;
      }
    }
    sm.dst[tid] = dst;
    sm.L[tid] = L;
    sm.M[tid] = mflag;
    sm.lit[tid] = litk;
    sm.O[tid] = O;
    __syncthreads();
    const uint32_t cnt = (n_seq - t0) < kTile ? (n_seq - t0) : kTile;
    const uint32_t d0 = carry_pos;
    const uint64_t d1w = (uint64_t)carry_pos + tp;
    const uint32_t d1 = d1w < blen ? (uint32_t)d1w : blen;
    for (uint32_t p0 = d0 + tid; p0 < d1; p0 += kTile) {
      uint32_t p = p0;
      uint8_t v = 0;
      for (;;) {
        const uint32_t s = find_seq(sm.dst, cnt, p);
        const uint32_t r = p - sm.dst[s];
        const uint32_t Ls = sm.L[s];
        if (r < Ls) {
          uint32_t li = sm.lit[s] + r;
          v = li < n_lit ? lit[li] : 0;
          break;
        }
        const uint32_t Ms = sm.M[s];
        if (Ms & kPoison) break;
        const uint32_t ii = r - Ls;
        const uint64_t mabs = bs + sm.dst[s] + Ls;
        const uint64_t Os = sm.O[s];
        const uint64_t dist = mabs - Os;
        const uint64_t src = Os + (ii < dist ? ii : (uint64_t)(ii % (uint32_t)dist));
        if (src < bs) {
          const uint64_t c = src / a.B;
          v = reinterpret_cast<const uint8_t*>(a.loc[c])[src - c * a.B];
          n_ext++;
          break;
        }
        const uint32_t q = (uint32_t)(src - bs);
        if (q < d0) {
          v = out[q];
          break;
        }
        p = q;
      }
      out[p0] = v;
    }
    carry_pos = (uint32_t)((uint64_t)carry_pos + tp > 0xFFFFFFFFull ? 0xFFFFFFFFu : carry_pos + tp);
    carry_lit += tl;
    if ((uint64_t)carry_pos > blen) bad = true;
    __syncthreads();
    if ((uint64_t)carry_pos >= blen) {
      if (t0 + kTile < n_seq) bad = true;  // sequences beyond the block end
      break;
    }
  }
  if (tid == 0 && (carry_pos != blen || carry_lit > n_lit)) bad = true;
  if (bad) flag(a.err, kErrCorrupt);
  n_ext = wave_total(n_ext);
  if ((tid & 63) == 0 && n_ext) atomicAdd(a.ext_bytes, (unsigned long long)n_ext);
}

__global__ __launch_bounds__(256) void k_expand(DecodeArgs a, uint32_t plan_lo) {
  __shared__ ExpandSmem<256> sm;
  expand_block<256>(a, plan_lo + blockIdx.x, sm);
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
  for (;;) {
    uint32_t i = 0;
    if (lane == 0) i = atomicAdd(a.queue, 1u);
    i = __shfl(i, 0, 64);
    if (i >= a.n_plan) break;
    const PlanEntry pe = a.plan[i];
    if (lane == 0) a.loc[pe.block] = a.dst_base + pe.dst;
    decode_stream(a, pe, i, 1, rs, lane);
    decode_stream(a, pe, i, 2, rs, lane);
    decode_stream(a, pe, i, 0, rs, lane);
    // dependencies: every listed earlier block must have published
    const uint8_t* be = a.arch + kHdr + (uint64_t)kBlk * pe.block;
    const uint32_t dep_off = ld32(be + 20), dep_cnt = ld32(be + 24);
    const uint32_t* deps = reinterpret_cast<const uint32_t*>(a.arch + kHdr + (uint64_t)kBlk * a.n_blocks) + dep_off;
    bool timeout = false;
    for (uint32_t j = lane; j < dep_cnt; j += kWave) {
      uint32_t* f = a.done + deps[j];
      uint32_t spins = 0;
      while (__hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != a.epoch) {
        if (++spins > a.spin_limit) {
          timeout = true;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    if (__ballot(timeout) && lane == 0) flag(a.err, kErrTimeout);
    __syncthreads();  // streams of this block written, dependencies visible to all lanes
    expand_block<64>(a, i, es);
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
  hipLaunchKernelGGL(k_expand, dim3(hi - lo), dim3(256), 0, s, a, lo);
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
