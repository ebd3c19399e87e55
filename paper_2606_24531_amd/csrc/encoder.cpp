// Host encoder of libaceseek (the paper's encoder runs on the CPU; Section 2:
// a global match search whose back-references are absolute output positions,
// with the output cut into fixed-size blocks).
//
// Policy (encoder-only; any legal parse decodes the same):
//   hash of X[p .. p+k): h = sum X[p+i] * 0x01000193^(k-1-i) mod 2^32,
//   bucket = (h * 0x9E3779B1 mod 2^32) >> (32 - hbits),
//   hbits = clamp(ceil(log2 n), 12, 27); chains link each position to the
//   previous one of its bucket.  At p the chain is walked most recent first
//   for at most max_chain candidates; a candidate's length is its common
//   prefix with p (overlap allowed) capped at the block end and 65535.
//   Longest wins, ties to the first found; taken if it reaches
//   min_match.  With a level cap, blocks are grouped in epochs of 64 (E in
//   all), counted in units of c = max(1, floor(E / 64)) epochs: a block of
//   epoch e takes sources only from itself and from blocks of earlier epochs
//   whose level is below min(cap - 1, floor(log2(floor(e / c) + 1)),
//   max(1, floor(log2(floor(E / c) + 1)) - 1)), so levels stay below the cap
//   and grow geometrically in size; chain candidates elsewhere are passed over without
//   being counted (at most 8 * max_chain chain steps), and a counted
//   candidate is cut where its source first enters such a block.
//   Frequencies are normalised to 4096 with f = max(1,
//   floor(c*4096/n)), the deficit added to the largest f (ties: lower
//   symbol) and any excess taken one at a time from the largest f > 1.
//
// Speed-ups that leave the parse unchanged: a rolling hash; chains built in
// parallel by bucket range; a candidate is skipped unless it matches at the
// current best length (it could not be strictly longer); the walk stops once
// a candidate reaches the longest possible length; blocks are parsed in
// parallel (with a level cap, the blocks of one epoch in parallel: they depend
// only on the final levels of earlier epochs).
#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/aceseek.h"
#include "common.h"

namespace {

thread_local std::string g_enc_err;

int efail(int code, const char* fmt, ...);

struct Seq {
  uint32_t L, M;
  uint64_t O;
};

inline void put16(uint8_t* p, uint32_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); }
inline void put32(uint8_t* p, uint32_t v) { for (int i = 0; i < 4; i++) p[i] = (uint8_t)(v >> (8 * i)); }
inline void put64(uint8_t* p, uint64_t v) { for (int i = 0; i < 8; i++) p[i] = (uint8_t)(v >> (8 * i)); }
inline uint64_t rup(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

uint32_t hash_bits(uint64_t n) {
  uint32_t b = 0;
  while (b < 63 && (1ull << b) < n) b++;
  return std::min<uint32_t>(27, std::max<uint32_t>(12, b));
}

unsigned thread_count(uint32_t want) {
  unsigned hw = std::thread::hardware_concurrency();
  if (hw == 0) hw = 1;
  return want ? want : hw;
}

template <class F>
void parallel_for(uint64_t n, unsigned threads, F&& f) {
  if (threads <= 1 || n < 2) {
    for (uint64_t i = 0; i < n; i++) f(i);
    return;
  }
  std::atomic<uint64_t> next{0};
  std::vector<std::thread> pool;
  for (unsigned t = 0; t < threads; t++)
    pool.emplace_back([&] {
      for (uint64_t i; (i = next.fetch_add(1)) < n;) f(i);
    });
  for (auto& th : pool) th.join();
}

// ---------------------------------------------------------------------------
// hash chains
// ---------------------------------------------------------------------------
struct Chains {
  std::vector<uint32_t> prev;  // UINT32_MAX = none (positions < 2^32)
};

void build_chains(const uint8_t* x, uint64_t n, uint32_t k, unsigned threads, Chains& C) {
  const uint32_t hb = hash_bits(n);
  C.prev.assign(n, UINT32_MAX);
  if (n < k) return;
  const uint64_t npos = n - k + 1;
  // bucket of every hashed position, in parallel over slices (rolling hash)
  std::vector<uint32_t> bk(npos);
  uint32_t pk1 = 1;  // P^(k-1)
  for (uint32_t i = 0; i + 1 < k; i++) pk1 *= 0x01000193u;
  const uint64_t slice = 1 << 20;
  parallel_for((npos + slice - 1) / slice, threads, [&](uint64_t s) {
    uint64_t q0 = s * slice, q1 = std::min(npos, q0 + slice);
    uint32_t h = 0;
    for (uint32_t i = 0; i < k; i++) h = h * 0x01000193u + x[q0 + i];
    for (uint64_t q = q0; q < q1; q++) {
      bk[q] = (uint32_t)(h * 0x9E3779B1u) >> (32 - hb);
      if (q + k < n) h = (h - x[q] * pk1) * 0x01000193u + x[q + k];
    }
  });
  // link: each thread owns a range of buckets and scans every position
  const unsigned T = std::max(1u, std::min(threads, 64u));
  const uint64_t nbk = 1ull << hb;
  parallel_for(T, T, [&](uint64_t t) {
    const uint32_t lo = (uint32_t)(nbk * t / T), hi = (uint32_t)(nbk * (t + 1) / T);
    std::vector<uint32_t> head(hi - lo, UINT32_MAX);
    for (uint64_t q = 0; q < npos; q++) {
      const uint32_t b = bk[q];
      if (b < lo || b >= hi) continue;
      C.prev[q] = head[b - lo];
      head[b - lo] = (uint32_t)q;
    }
  });
}

inline uint32_t common_prefix(const uint8_t* a, const uint8_t* b, uint32_t lim) {
  uint32_t i = 0;
  while (i + 8 <= lim) {
    uint64_t u, v;
    memcpy(&u, a + i, 8);
    memcpy(&v, b + i, 8);
    if (u != v) return i + (uint32_t)(__builtin_ctzll(u ^ v) >> 3);
    i += 8;
  }
  while (i < lim && a[i] == b[i]) i++;
  return i;
}

// ---------------------------------------------------------------------------
// parse
// ---------------------------------------------------------------------------
struct ParseCtx {
  const uint8_t* x;
  uint64_t n;
  const ace_encode_params* p;
  const Chains* C;
  // level cap: sorted blocks of earlier epochs at or above the epoch's level budget
  const std::vector<uint32_t>* deep;
};

uint32_t level_budget(uint64_t e, uint64_t n_ep, uint32_t cap) {
  auto lg = [](uint64_t v) {
    uint32_t r = 0;
    while (v >>= 1) r++;
    return r;
  };
  const uint64_t c = std::max<uint64_t>(1, n_ep / 64);
  const uint32_t top = std::max<uint32_t>(1, lg(n_ep / c + 1) >= 1 ? lg(n_ep / c + 1) - 1 : 0);
  return std::min({lg(e / c + 1), top, cap - 1});
}

void push_seq(std::vector<Seq>& out, uint64_t lits, uint32_t M, uint64_t O) {
  while (lits > 65535) {
    out.push_back(Seq{65535, 0, 0});
    lits -= 65535;
  }
  out.push_back(Seq{(uint32_t)lits, M, O});
}

void parse_block(const ParseCtx& c, uint64_t b, bool capped, std::vector<Seq>& out) {
  const uint64_t B = c.p->block_size, s = b * B, e = std::min(s + B, c.n);
  const uint32_t mm = c.p->min_match, k = c.p->hash_len;
  uint64_t pos = s, lit0 = s;
  out.clear();
  while (pos < e) {
    uint32_t best = 0;
    uint64_t bestq = 0;
    if (pos + k <= c.n && e - pos >= mm) {
      const uint32_t lim = (uint32_t)std::min<uint64_t>(e - pos, 65535);
      uint32_t q = c.C->prev[pos];
      const uint64_t ep_lo = capped ? (b / 64) * 64 * B : s;
      uint32_t steps = 0;
      for (uint32_t cand = 0; q != UINT32_MAX && cand < c.p->max_chain && steps < 8 * c.p->max_chain;
           steps++, q = c.C->prev[q]) {
        if (capped && q < s &&
            (q >= ep_lo || std::binary_search(c.deep->begin(), c.deep->end(), (uint32_t)(q / B))))
          continue;  // starts in an invisible block: passed over, not counted
        cand++;
        // only a candidate agreeing at offset `best` can be strictly longer
        if (best && c.x[q + best] != c.x[pos + best]) continue;
        uint32_t len = common_prefix(c.x + q, c.x + pos, lim);
        if (len <= best) continue;
        if (capped) {
          const uint64_t end = std::min<uint64_t>((uint64_t)q + len, s);
          if ((uint64_t)q < end) {
            const auto& d = *c.deep;
            auto it = std::lower_bound(d.begin(), d.end(), (uint32_t)(q / B));
            uint64_t cut = it != d.end() ? (uint64_t)*it * B : UINT64_MAX;
            if (ep_lo < s) cut = std::min(cut, ep_lo);
            if (cut < end) len = cut > q ? (uint32_t)(cut - q) : 0;
          }
          if (len <= best) continue;
        }
        best = len;
        bestq = q;
        if (best == lim) break;
      }
    }
    if (best >= mm) {
      push_seq(out, pos - lit0, best, bestq);
      pos += best;
      lit0 = pos;
    } else {
      pos++;
    }
  }
  if (lit0 < e) push_seq(out, e - lit0, 0, 0);
}

// Blocks the block's matches read before the block start, sorted, unique.
void deps_of(const std::vector<Seq>& seqs, uint64_t b, uint64_t B, std::vector<uint32_t>& d) {
  d.clear();
  const uint64_t bs = b * B;
  for (const Seq& q : seqs) {
    if (!q.M) continue;
    const uint64_t end = std::min<uint64_t>(q.O + q.M, bs);
    for (uint64_t a = q.O; a < end; a = (a / B + 1) * B) d.push_back((uint32_t)(a / B));
  }
  std::sort(d.begin(), d.end());
  d.erase(std::unique(d.begin(), d.end()), d.end());
}

// ---------------------------------------------------------------------------
// entropy coding of one stream
// ---------------------------------------------------------------------------
void normalise(const uint64_t* cnt, uint64_t n, uint32_t* f) {
  int64_t sum = 0;
  for (int s = 0; s < 256; s++) {
    f[s] = cnt[s] ? std::max<uint64_t>(1, cnt[s] * 4096 / n) : 0;
    sum += f[s];
  }
  auto largest = [&](uint32_t floor_) {
    int best = -1;
    for (int s = 0; s < 256; s++)
      if (f[s] > floor_ && (best < 0 || f[s] > f[best])) best = s;
    return best;
  };
  if (sum < 4096) f[largest(0)] += (uint32_t)(4096 - sum);
  while (sum > 4096) {
    f[largest(1)]--;
    sum--;
  }
}

struct EncStream {
  uint8_t mode = 0;
  uint32_t n_sym = 0;
  std::vector<uint8_t> data;
};

void code_stream(const uint8_t* sym, uint32_t n, uint32_t W, uint32_t policy, EncStream& es) {
  es.n_sym = n;
  es.mode = 0;
  es.data.assign(sym, sym + n);
  if (n == 0 || policy == 2) return;
  uint64_t cnt[256] = {0};
  for (uint32_t i = 0; i < n; i++) cnt[sym[i]]++;
  uint32_t f[256], cum[256];
  normalise(cnt, n, f);
  uint32_t present = 0, c = 0;
  for (int s = 0; s < 256; s++) {
    cum[s] = c;
    c += f[s];
    present += f[s] != 0;
  }
  const uint32_t tsz = (32 + 2 * present + 3) & ~3u;
  // words are produced last-symbol first; at most one per symbol
  std::vector<uint16_t> words;
  words.reserve(n / 2 + 16);
  uint32_t x[64];
  for (uint32_t j = 0; j < W; j++) x[j] = 65536;
  for (uint32_t i = n; i-- > 0;) {
    const uint32_t j = i % W, fs = f[sym[i]];
    if ((uint64_t)x[j] >= ((uint64_t)fs << 20)) {
      words.push_back((uint16_t)x[j]);
      x[j] >>= 16;
    }
    x[j] = (x[j] / fs) * 4096 + (x[j] % fs) + cum[sym[i]];
  }
  const uint64_t size = tsz + 4ull * W + 2ull * words.size();
  if (policy != 1 && size >= n) return;
  es.mode = 1;
  es.data.assign(size, 0);
  uint8_t* o = es.data.data();
  uint8_t* fp = o + 32;
  for (int s = 0; s < 256; s++)
    if (f[s]) {
      o[s >> 3] |= (uint8_t)(1u << (s & 7));
      put16(fp, f[s] - 1);
      fp += 2;
    }
  for (uint32_t j = 0; j < W; j++) put32(o + tsz + 4 * j, x[j]);
  uint8_t* wp = o + tsz + 4 * W;
  for (size_t i = 0; i < words.size(); i++) put16(wp + 2 * i, words[words.size() - 1 - i]);
}

// Bytes per stored absolute offset: 4 while every position fits in 32 bits,
// else 8; ACE_ENC_WIDE_OFFSETS asks for 8 at any size.
uint32_t offset_width(uint64_t n, uint32_t flags) {
  return (n > (1ull << 32) || (flags & ACE_ENC_WIDE_OFFSETS)) ? 8u : 4u;
}

// The rANS step of every stream on the current device (the streams built,
// each holding its raw symbols): one wavefront per stream, the same bytes
// as code_stream.  Streams the device codes take mode 1 and the coded bytes.
int device_entropy(std::vector<EncStream>& st, uint32_t W, uint32_t policy) {
  const size_t ns = st.size();
  if (ns == 0) return ACE_OK;
  std::vector<uint64_t> sym_off(ns), out_off(ns), scr_off(ns);
  std::vector<uint32_t> nsym(ns);
  uint64_t a = 0, o = 0, w = 0;
  for (size_t i = 0; i < ns; i++) {
    nsym[i] = st[i].n_sym;
    sym_off[i] = a;
    out_off[i] = o;
    scr_off[i] = w;
    a += st[i].n_sym;
    o += rup(544 + 4ull * W + 2ull * st[i].n_sym, 16);
    w += st[i].n_sym;
  }
  std::vector<uint8_t> sym(a ? a : 1);
  for (size_t i = 0; i < ns; i++)
    if (st[i].n_sym) memcpy(sym.data() + sym_off[i], st[i].data.data(), st[i].n_sym);
  uint8_t *d_sym = nullptr, *d_out = nullptr;
  uint64_t *d_soff = nullptr, *d_ooff = nullptr, *d_woff = nullptr;
  uint32_t *d_n = nullptr, *d_len = nullptr;
  uint16_t* d_scr = nullptr;
  auto release = [&]() {
    for (void* q : {(void*)d_sym, (void*)d_out, (void*)d_soff, (void*)d_ooff, (void*)d_woff, (void*)d_n,
                    (void*)d_len, (void*)d_scr})
      if (q) (void)hipFree(q);
  };
  auto hip = [&](hipError_t r, const char* what) {
    if (r == hipSuccess) return ACE_OK;
    release();
    return efail(ACE_E_HIP, "device entropy coding: %s: %s", what, hipGetErrorString(r));
  };
  int rc;
  if ((rc = hip(hipMalloc((void**)&d_sym, sym.size()), "allocate symbols")) ||
      (rc = hip(hipMalloc((void**)&d_out, o ? o : 16), "allocate output")) ||
      (rc = hip(hipMalloc((void**)&d_scr, 2 * (w ? w : 1)), "allocate scratch")) ||
      (rc = hip(hipMalloc((void**)&d_soff, 8 * ns), "allocate offsets")) ||
      (rc = hip(hipMalloc((void**)&d_ooff, 8 * ns), "allocate offsets")) ||
      (rc = hip(hipMalloc((void**)&d_woff, 8 * ns), "allocate offsets")) ||
      (rc = hip(hipMalloc((void**)&d_n, 4 * ns), "allocate counts")) ||
      (rc = hip(hipMalloc((void**)&d_len, 4 * ns), "allocate lengths")))
    return rc;
  if ((rc = hip(hipMemcpy(d_sym, sym.data(), sym.size(), hipMemcpyHostToDevice), "copy symbols")) ||
      (rc = hip(hipMemcpy(d_soff, sym_off.data(), 8 * ns, hipMemcpyHostToDevice), "copy offsets")) ||
      (rc = hip(hipMemcpy(d_ooff, out_off.data(), 8 * ns, hipMemcpyHostToDevice), "copy offsets")) ||
      (rc = hip(hipMemcpy(d_woff, scr_off.data(), 8 * ns, hipMemcpyHostToDevice), "copy offsets")) ||
      (rc = hip(hipMemcpy(d_n, nsym.data(), 4 * ns, hipMemcpyHostToDevice), "copy counts")))
    return rc;
  ace::EncArgs e{};
  e.sym = d_sym;
  e.sym_off = d_soff;
  e.n = d_n;
  e.out = d_out;
  e.out_off = d_ooff;
  e.scratch = d_scr;
  e.scr_off = d_woff;
  e.out_len = d_len;
  e.W = W;
  e.policy = policy;
  e.n_streams = (uint32_t)ns;
  if ((rc = hip(ace::launch_rans_encode(e, nullptr), "launch")) || (rc = hip(hipDeviceSynchronize(), "run")))
    return rc;
  std::vector<uint32_t> len(ns);
  std::vector<uint8_t> out(o ? o : 16);
  if ((rc = hip(hipMemcpy(len.data(), d_len, 4 * ns, hipMemcpyDeviceToHost), "copy lengths")) ||
      (rc = hip(hipMemcpy(out.data(), d_out, out.size(), hipMemcpyDeviceToHost), "copy output")))
    return rc;
  release();
  for (size_t i = 0; i < ns; i++) {
    if (!len[i]) continue;  // stays raw
    st[i].mode = 1;
    st[i].data.assign(out.data() + out_off[i], out.data() + out_off[i] + len[i]);
  }
  return ACE_OK;
}

int check(uint64_t n, const ace_encode_params* p) {
  if (!p) return efail(ACE_E_ARG, "null parameters");
  if (p->block_size < 1 || p->block_size > (1u << 24)) return efail(ACE_E_ARG, "block_size outside 1..2^24");
  if (p->interleave < 1 || p->interleave > 64) return efail(ACE_E_ARG, "interleave outside 1..64");
  if (p->hash_len < 1 || p->hash_len > 64) return efail(ACE_E_ARG, "hash_len outside 1..64");
  if (p->min_match < p->hash_len) return efail(ACE_E_ARG, "min_match below hash_len");
  if ((p->flags & 3) == 3) return efail(ACE_E_ARG, "unknown stream-mode policy");
  if (p->flags & ~15u) return efail(ACE_E_ARG, "unknown flag bits 0x%x", p->flags & ~15u);
  if (n > (1ull << 32)) return efail(ACE_E_ARG, "inputs above 4 GiB are not supported by this encoder");
  return ACE_OK;
}

}  // namespace

// host.cpp owns the message buffer behind ace_last_error(); the encoder
// reports through the same thread-local channel via this hook.
extern "C" void ace_internal_set_error(const char* msg);

namespace {
int efail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  ace_internal_set_error(buf);
  return code;
}
}  // namespace

extern "C" int ace_encode_bound(uint64_t n, const ace_encode_params* p, uint64_t* bound) {
  int rc = check(n, p);
  if (rc) return rc;
  if (!bound) return efail(ACE_E_ARG, "null bound");
  const uint64_t B = p->block_size, nb = n ? (n + B - 1) / B : 0, W = p->interleave;
  uint64_t total = 64 + 32 * nb + 16;
  for (uint64_t b = 0; b < nb; b++) {
    const uint64_t len = std::min<uint64_t>(B, n - b * B);
    uint64_t nseq = std::min<uint64_t>(len, len / p->min_match + len / 65535 + 2);
    const uint64_t dep = std::min<uint64_t>(b, 2 * nseq + 1);
    const uint64_t syms[3] = {len, 4 * nseq, offset_width(n, p->flags) * nseq};
    uint64_t sz = 16 + 48 + 4 * dep;
    for (int t = 0; t < 3; t++) sz += 3 + ((p->flags & 3) == 1 ? 544 + 4 * W + 2 * syms[t] : syms[t]);
    total += sz;
  }
  *bound = total;
  return ACE_OK;
}

extern "C" int ace_encode_archive(const uint8_t* x, uint64_t n, const ace_encode_params* p,
                                  uint8_t* dst, uint64_t cap, uint64_t* out_len) {
  int rc = check(n, p);
  if (rc) return rc;
  if ((!x && n) || !out_len) return efail(ACE_E_ARG, "null argument");
  const unsigned T = thread_count(p->n_threads);
  const uint64_t B = p->block_size, nb = n ? (n + B - 1) / B : 0;
  const uint32_t W = p->interleave, policy = p->flags & 3, ow = offset_width(n, p->flags);
  Chains C;
  // optional progress lines on stderr (environment ACESEEK_ENCODE_PROGRESS=1),
  // for callers that must show a long encode is alive
  const char* pe = getenv("ACESEEK_ENCODE_PROGRESS");
  const bool progress = pe && pe[0] == '1';
  std::atomic<uint64_t> parsed{0};
  auto report = [&](uint64_t done_blocks) {
    if (progress && nb >= 16 && done_blocks % ((nb + 15) / 16) == 0)
      fprintf(stderr, "[aceseek encode] parsed %llu of %llu blocks\n", (unsigned long long)done_blocks,
              (unsigned long long)nb), fflush(stderr);
  };
  build_chains(x, n, p->hash_len, T, C);
  if (progress) fprintf(stderr, "[aceseek encode] hash chains built (%llu bytes)\n", (unsigned long long)n), fflush(stderr);
  std::vector<std::vector<Seq>> seqs(nb);
  std::vector<uint32_t> level(nb, 0);
  std::vector<std::vector<uint32_t>> deps(nb);
  std::vector<uint32_t> deep;
  ParseCtx pc{x, n, p, &C, &deep};
  if (p->max_level) {
    // epochs of 64 blocks: blocks of one epoch see only earlier epochs, below
    // the epoch's level budget
    const uint64_t n_ep = (nb + 63) / 64;
    uint32_t lam = 0;
    for (uint64_t e0 = 0; e0 < nb; e0 += 64) {
      const uint64_t e1 = std::min<uint64_t>(nb, e0 + 64);
      const uint32_t l = level_budget(e0 / 64, n_ep, p->max_level);
      if (l != lam) {  // the budget only grows: drop blocks that became visible
        lam = l;
        deep.erase(std::remove_if(deep.begin(), deep.end(), [&](uint32_t b) { return level[b] < lam; }),
                   deep.end());
      }
      parallel_for(e1 - e0, T, [&](uint64_t i) {
        parse_block(pc, e0 + i, true, seqs[e0 + i]);
        report(++parsed);
      });
      for (uint64_t b = e0; b < e1; b++) {
        deps_of(seqs[b], b, B, deps[b]);
        uint32_t lv = 0;
        for (uint32_t d : deps[b]) lv = std::max(lv, level[d] + 1);
        level[b] = lv;
        if (lv >= lam) deep.push_back((uint32_t)b);
      }
    }
  } else {
    parallel_for(nb, T, [&](uint64_t b) {
      parse_block(pc, b, false, seqs[b]);
      report(++parsed);
    });
    for (uint64_t b = 0; b < nb; b++) {
      deps_of(seqs[b], b, B, deps[b]);
      uint32_t lv = 0;
      for (uint32_t d : deps[b]) lv = std::max(lv, level[d] + 1);
      level[b] = lv;
    }
  }
  std::vector<uint32_t>().swap(C.prev);
  // streams, in parallel over blocks
  std::vector<EncStream> st(3 * nb);
  const bool device = (p->flags & ACE_ENC_DEVICE_ENTROPY) != 0;
  parallel_for(nb, T, [&](uint64_t b) {
    const std::vector<Seq>& sq = seqs[b];
    std::vector<uint8_t> lit, lens(4 * sq.size()), offs(ow * sq.size());
    uint64_t pos = b * B;
    for (size_t k = 0; k < sq.size(); k++) {
      lit.insert(lit.end(), x + pos, x + pos + sq[k].L);
      pos += sq[k].L + sq[k].M;
      put16(&lens[4 * k], sq[k].L);
      put16(&lens[4 * k + 2], sq[k].M);
      for (uint32_t i = 0; i < ow; i++) offs[ow * k + i] = (uint8_t)(sq[k].O >> (8 * i));
    }
    if (device) {  // raw for now: coded on the device below
      const std::vector<uint8_t>* v[3] = {&lit, &lens, &offs};
      for (int t = 0; t < 3; t++) {
        st[3 * b + t].n_sym = (uint32_t)v[t]->size();
        st[3 * b + t].data = *v[t];
      }
      return;
    }
    code_stream(lit.data(), (uint32_t)lit.size(), W, policy, st[3 * b]);
    code_stream(lens.data(), (uint32_t)lens.size(), W, policy, st[3 * b + 1]);
    code_stream(offs.data(), (uint32_t)offs.size(), W, policy, st[3 * b + 2]);
  });
  if (device && (rc = device_entropy(st, W, policy))) return rc;
  // layout
  uint64_t n_deps = 0, depth = 0;
  for (uint64_t b = 0; b < nb; b++) {
    n_deps += deps[b].size();
    depth = std::max<uint64_t>(depth, level[b] + 1);
  }
  const uint64_t deps_at = 64 + 32 * nb, pay_at = rup(deps_at + 4 * n_deps, 16);
  std::vector<uint64_t> pay(nb);
  uint64_t at = pay_at;
  for (uint64_t b = 0; b < nb; b++) {
    at = rup(at, 16);
    pay[b] = at;
    uint64_t sz = 48;
    for (int t = 0; t < 3; t++) sz = rup(sz, 4) + st[3 * b + t].data.size();
    at += sz;
  }
  *out_len = at;
  if (!dst || cap < at) return efail(ACE_E_NOSPACE, "archive needs %llu bytes", (unsigned long long)at);
  memset(dst, 0, pay_at);
  put32(dst, 0x314B5341u);
  put16(dst + 4, 1);
  put32(dst + 8, (uint32_t)B);
  put16(dst + 12, (uint16_t)W);
  dst[14] = 12;
  dst[15] = (uint8_t)ow;
  put64(dst + 16, n);
  put32(dst + 24, (uint32_t)nb);
  put32(dst + 28, (uint32_t)depth);
  put32(dst + 32, p->max_level);
  put32(dst + 36, (uint32_t)n_deps);
  put64(dst + 40, 64);
  put64(dst + 48, pay_at);
  uint64_t h = 0xcbf29ce484222325ull;
  for (uint64_t i = 0; i < n; i++) h = (h ^ x[i]) * 0x100000001b3ull;
  put64(dst + 56, h);
  uint64_t di = 0;
  for (uint64_t b = 0; b < nb; b++) {
    uint8_t* e = dst + 64 + 32 * b;
    const uint64_t plen_end = (b + 1 < nb ? pay[b + 1] : at);
    put64(e, pay[b]);
    put32(e + 12, (uint32_t)seqs[b].size());
    put32(e + 16, level[b]);
    put32(e + 20, (uint32_t)di);
    put32(e + 24, (uint32_t)deps[b].size());
    for (uint32_t d : deps[b]) put32(dst + deps_at + 4 * (di++), d);
    (void)plen_end;
  }
  parallel_for(nb, T, [&](uint64_t b) {
    uint8_t* pl = dst + pay[b];
    uint64_t off = 48;
    for (int t = 0; t < 3; t++) {
      const EncStream& es = st[3 * b + t];
      const uint64_t o = rup(off, 4);
      memset(pl + off, 0, o - off);
      uint8_t* d = pl + 16 * t;
      memset(d, 0, 16);
      d[0] = es.mode;
      put32(d + 4, es.n_sym);
      put32(d + 8, (uint32_t)es.data.size());
      put32(d + 12, (uint32_t)o);
      memcpy(pl + o, es.data.data(), es.data.size());
      off = o + es.data.size();
    }
    put32(dst + 64 + 32 * b + 8, (uint32_t)off);
    const uint64_t next = b + 1 < nb ? pay[b + 1] : at;
    memset(pl + off, 0, next - (pay[b] + off));
  });
  return ACE_OK;
}
