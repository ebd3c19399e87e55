// Host side of libaceseek: archive validation, the seek planner and the C
// ABI entry points declared in include/aceseek.h.
//
// Planner (paper Sections 2, 3, 5 and 7).  A range [lo, hi) names target
// blocks floor(lo/B) .. floor((hi-1)/B).  Because every back-reference is an
// absolute position, a block can be decoded as soon as every earlier block
// its matches copy from is decoded; the index lists those blocks per block, so
// the set of blocks a seek needs is the closure of the targets under that
// relation, and a valid order is by increasing dependency level.  Target
// blocks that the range covers whole are decoded straight into the caller's
// output; every other block of the closure goes to a workspace slot, and the
// partial first and last blocks are clipped out of their slots afterwards.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/aceseek.h"
#include "common.h"

using namespace ace;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

inline uint16_t h16(const uint8_t* p) { return (uint16_t)(p[0] | (p[1] << 8)); }
inline uint32_t h32(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}
inline uint64_t h64(const uint8_t* p) { return (uint64_t)h32(p) | ((uint64_t)h32(p + 4) << 32); }
inline uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(ACE_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

}  // namespace

struct BlockInfo {
  uint32_t n_seq, level, dep_off, dep_cnt, n_lit, plen;
  uint64_t pay;
  uint64_t raw[3];  // archive offset of each stream's data when stored raw, else kCoded
};

struct ace_archive {
  const uint8_t* d_arch = nullptr;
  uint64_t len = 0, n = 0;
  uint32_t B = 0, W = 0, ow = 0, nb = 0, depth = 0;
  std::vector<BlockInfo> blk;
  std::vector<uint32_t> deps;
  // whole-archive plan: blocks by level, their token slots, level boundaries
  std::vector<PlanEntry> all_plan;
  std::vector<uint32_t> all_levels;
  uint64_t all_seq = 0;
  PlanEntry* all_plan_pinned = nullptr;
  const PlanEntry* d_plan = nullptr;  // the whole-archive plan resident on the device, if attached
  const uint32_t* d_order = nullptr;  // with it: all blocks by level, then the level boundaries
  const uint32_t* d_lstart = nullptr;
  std::mutex pin_mu;
  // out of core: the archive stays in host memory (h_arch, the caller's);
  // each seek stages what it needs through a pinned buffer
  const uint8_t* h_arch = nullptr;
  std::mutex ooc_mu;
  uint8_t* ooc_pinned = nullptr;
  uint64_t ooc_pinned_cap = 0;
  ~ace_archive() {
    if (all_plan_pinned) (void)hipHostFree(all_plan_pinned);
    if (ooc_pinned) (void)hipHostFree(ooc_pinned);
  }
};

// The entry points that read the archive on the device need it resident.
static int need_resident(const ace_archive* A) {
  if (A && !A->d_arch && A->h_arch)
    return fail(ACE_E_ARG, "the archive was opened out of core: its ranges decode with ace_seek_ooc");
  return ACE_OK;
}

static PlanEntry make_entry(const ace_archive* A, uint32_t b, uint64_t seq_base, uint64_t dst) {
  const BlockInfo& bi = A->blk[b];
  PlanEntry e{};
  e.block = b;
  e.seq_base = (uint32_t)seq_base;
  e.dst = dst;
  e.pay = bi.pay;
  e.n_seq = bi.n_seq;
  e.n_lit = bi.n_lit;
  e.dep_off = bi.dep_off;
  e.dep_cnt = bi.dep_cnt;
  for (int t = 0; t < 3; t++) e.raw[t] = bi.raw[t];
  return e;
}

extern "C" const char* ace_last_error(void) { return g_err.c_str(); }
extern "C" void ace_internal_set_error(const char* msg) { g_err = msg; }

// ---------------------------------------------------------------------------
// open / validate
// ---------------------------------------------------------------------------
static int validate(const uint8_t* a, uint64_t len, ace_archive* A) {
  if (len < kHdr) return fail(ACE_E_CORRUPT, "archive shorter than its 64-byte header");
  if (h32(a) != kMagic) return fail(ACE_E_CORRUPT, "bad magic");
  if (h16(a + 4) != 1) return fail(ACE_E_CORRUPT, "unsupported version %u", h16(a + 4));
  A->B = h32(a + 8);
  A->W = h16(a + 12);
  A->ow = a[15];
  A->n = h64(a + 16);
  A->nb = h32(a + 24);
  A->depth = h32(a + 28);
  const uint32_t max_level = h32(a + 32), n_deps = h32(a + 36);
  if (a[14] != kProbBits) return fail(ACE_E_CORRUPT, "probability bits %u (expected 12)", a[14]);
  if (A->B < 1 || A->B > (1u << 24)) return fail(ACE_E_CORRUPT, "block size %u out of range", A->B);
  if (A->W < 1 || A->W > 64) return fail(ACE_E_CORRUPT, "interleave %u out of range", A->W);
  if (A->ow != 4 && A->ow != 8) return fail(ACE_E_CORRUPT, "offset width %u", A->ow);
  if (A->ow == 4 && A->n > (1ull << 32)) return fail(ACE_E_CORRUPT, "4-byte offsets for more than 4 GiB");
  const uint64_t nb = A->n ? (A->n - 1) / A->B + 1 : 0;
  if (nb != A->nb) return fail(ACE_E_CORRUPT, "block count %u does not match ceil(N/B) = %llu", A->nb,
                               (unsigned long long)nb);
  if (h64(a + 40) != kHdr) return fail(ACE_E_CORRUPT, "block table must follow the header");
  const uint64_t deps_at = kHdr + (uint64_t)kBlk * A->nb, pay_at = h64(a + 48);
  if (deps_at + 4ull * n_deps > len || pay_at < deps_at + 4ull * n_deps || pay_at > len)
    return fail(ACE_E_CORRUPT, "index does not fit the archive");
  A->deps.resize(n_deps);
  for (uint32_t i = 0; i < n_deps; i++) A->deps[i] = h32(a + deps_at + 4ull * i);
  A->blk.resize(A->nb);
  uint32_t max_lv_plus1 = 0;
  for (uint32_t b = 0; b < A->nb; b++) {
    const uint8_t* e = a + kHdr + (uint64_t)kBlk * b;
    const uint64_t pay = h64(e);
    const uint32_t plen = h32(e + 8);
    BlockInfo& bi = A->blk[b];
    bi.n_seq = h32(e + 12);
    bi.level = h32(e + 16);
    bi.dep_off = h32(e + 20);
    bi.dep_cnt = h32(e + 24);
    bi.pay = pay;
    bi.plen = plen;
    if (h32(e + 28) != 0) return fail(ACE_E_CORRUPT, "block %u: reserved field is not zero", b);
    if (pay % 16 || pay < pay_at || pay + plen > len || plen < 3 * kSDesc)
      return fail(ACE_E_CORRUPT, "block %u: payload outside the archive", b);
    const uint64_t bs = (uint64_t)b * A->B;
    const uint32_t blen = (uint32_t)std::min<uint64_t>(A->B, A->n - bs);
    if (bi.n_seq == 0 || bi.n_seq > blen) return fail(ACE_E_CORRUPT, "block %u: %u sequences", b, bi.n_seq);
    if ((uint64_t)bi.dep_off + bi.dep_cnt > n_deps)
      return fail(ACE_E_CORRUPT, "block %u: dependency list outside the index", b);
    uint32_t lv = 0;
    for (uint32_t j = 0; j < bi.dep_cnt; j++) {
      const uint32_t d = A->deps[bi.dep_off + j];
      if (d >= b) return fail(ACE_E_CORRUPT, "block %u: dependency %u is not an earlier block", b, d);
      if (j && d <= A->deps[bi.dep_off + j - 1])
        return fail(ACE_E_CORRUPT, "block %u: dependencies not strictly ascending", b);
      lv = std::max(lv, A->blk[d].level + 1);
    }
    if (lv != bi.level) return fail(ACE_E_CORRUPT, "block %u: level %u, dependencies give %u", b, bi.level, lv);
    max_lv_plus1 = std::max(max_lv_plus1, lv + 1);
    const uint32_t want[3] = {0, 4 * bi.n_seq, A->ow * bi.n_seq};
    for (int t = 0; t < 3; t++) {
      const uint8_t* d = a + pay + kSDesc * t;
      const uint32_t mode = d[0], nsym = h32(d + 4), clen = h32(d + 8), off = h32(d + 12);
      if (d[1] | d[2] | d[3]) return fail(ACE_E_CORRUPT, "block %u stream %d: padding not zero", b, t);
      if (mode > 1) return fail(ACE_E_CORRUPT, "block %u stream %d: unknown mode %u", b, t, mode);
      if (off % 4 || off < 3 * kSDesc || (uint64_t)off + clen > plen)
        return fail(ACE_E_CORRUPT, "block %u stream %d: data outside the payload", b, t);
      if (t == 0 ? nsym > blen : nsym != want[t])
        return fail(ACE_E_CORRUPT, "block %u stream %d: %u symbols", b, t, nsym);
      if (mode == 0 && clen != nsym) return fail(ACE_E_CORRUPT, "block %u stream %d: raw size mismatch", b, t);
      if (mode == 1 && (nsym == 0 || clen < 36 + 4 * A->W))
        return fail(ACE_E_CORRUPT, "block %u stream %d: rANS stream too short", b, t);
      bi.raw[t] = mode == 0 ? pay + off : kCoded;
      if (t == 0) bi.n_lit = nsym;
    }
  }
  if (max_lv_plus1 != A->depth)
    return fail(ACE_E_CORRUPT, "stored depth %u, levels give %u", A->depth, max_lv_plus1);
  if (max_level && A->depth > max_level)
    return fail(ACE_E_CORRUPT, "depth %u exceeds the stated level cap %u", A->depth, max_level);
  A->len = len;
  return ACE_OK;
}

// Level order of a set of blocks (counting sort by level).  Within a level
// the blocks with more sequences come first (then by block id): a block's
// expansion time grows with its sequence count, and starting the long ones
// first keeps a level's last residency wave short (longest-first list
// scheduling).
static void level_order(const ace_archive* A, const std::vector<uint32_t>& blocks,
                        std::vector<uint32_t>& order, std::vector<uint32_t>& lstart) {
  lstart.assign(A->depth + 1, 0);
  for (uint32_t b : blocks) lstart[A->blk[b].level + 1]++;
  for (uint32_t l = 0; l < A->depth; l++) lstart[l + 1] += lstart[l];
  std::vector<uint32_t> pos(lstart.begin(), lstart.end() - 1);
  order.resize(blocks.size());
  for (uint32_t b : blocks) order[pos[A->blk[b].level]++] = b;
  std::vector<uint64_t> key;
  for (uint32_t l = 0; l < A->depth; l++) {
    const uint32_t lo = lstart[l], hi = lstart[l + 1];
    if (hi - lo < 2) continue;
    key.resize(hi - lo);
    for (uint32_t i = lo; i < hi; i++)
      key[i - lo] = ((uint64_t)(0xFFFFFFFFu - A->blk[order[i]].n_seq) << 32) | order[i];
    std::sort(key.begin(), key.end());
    for (uint32_t i = lo; i < hi; i++) order[i] = (uint32_t)key[i - lo];
  }
}

extern "C" int ace_archive_open(const uint8_t* h_arch, uint64_t len, const void* d_arch,
                                ace_archive** out) {
  if (!h_arch || !out) return fail(ACE_E_ARG, "null argument");
  ace_archive* A = new (std::nothrow) ace_archive();
  if (!A) return fail(ACE_E_NOMEM, "out of memory");
  int rc = validate(h_arch, len, A);
  if (rc) {
    delete A;
    return rc;
  }
  A->d_arch = static_cast<const uint8_t*>(d_arch);
  std::vector<uint32_t> all(A->nb), order;
  for (uint32_t b = 0; b < A->nb; b++) all[b] = b;
  level_order(A, all, order, A->all_levels);
  A->all_plan.resize(A->nb);
  uint64_t seq = 0;
  for (uint32_t i = 0; i < A->nb; i++) {
    const uint32_t b = order[i];
    A->all_plan[i] = make_entry(A, b, seq, (uint64_t)b * A->B);
    seq += A->blk[b].n_seq;
  }
  if (seq > 0xFFFFFFFFull) {
    delete A;
    return fail(ACE_E_CORRUPT, "more than 2^32 sequences");
  }
  A->all_seq = seq;
  *out = A;
  return ACE_OK;
}

extern "C" int ace_archive_open_ooc(const uint8_t* h_arch, uint64_t len, ace_archive** out) {
  if (!h_arch || !out) return fail(ACE_E_ARG, "null argument");
  ace_archive* A = nullptr;
  int rc = ace_archive_open(h_arch, len, nullptr, &A);
  if (rc) return rc;
  A->h_arch = h_arch;
  *out = A;
  return ACE_OK;
}

extern "C" void ace_archive_close(ace_archive* a) { delete a; }

extern "C" int ace_archive_info(const ace_archive* a, uint64_t* n_total, uint32_t* block_size,
                                uint32_t* n_blocks, uint32_t* depth) {
  if (!a) return fail(ACE_E_ARG, "null archive");
  if (n_total) *n_total = a->n;
  if (block_size) *block_size = a->B;
  if (n_blocks) *n_blocks = a->nb;
  if (depth) *depth = a->depth;
  return ACE_OK;
}

// ---------------------------------------------------------------------------
// planning and workspace layout
// ---------------------------------------------------------------------------
namespace {

// Optional phase timing (per thread): a pair of events around every entropy
// launch and every expansion launch of the last decode on this thread, each
// pair recorded on the stream the launch goes to.
struct PhaseTimer {
  bool on = false;
  std::vector<hipEvent_t> ent, mat;  // begin/end pairs
  size_t n_ent = 0, n_mat = 0;
  bool recorded = false;
  // host side of the last timed call: entry, then planning and enqueueing
  std::chrono::steady_clock::time_point t_enter;
  double us_plan = 0, us_enqueue = 0;
};
thread_local PhaseTimer g_timer;
inline void timer_enter() {
  if (g_timer.on) g_timer.t_enter = std::chrono::steady_clock::now();
}
inline double us_since(std::chrono::steady_clock::time_point t) {
  return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t).count();
}
// per-block clock trace of this thread's decodes (null: off)
thread_local unsigned long long* g_trace = nullptr;
thread_local uint64_t g_trace_entries = 0;

hipError_t timer_pair(std::vector<hipEvent_t>& v, size_t k) {
  while (v.size() < 2 * (k + 1)) {
    hipEvent_t e = nullptr;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    v.push_back(e);
  }
  return hipSuccess;
}

// The calling thread's second stream and level events on the current device:
// the entropy launches of later levels run on it beside the expansion of
// earlier levels on the caller's stream.
struct Overlap {
  hipStream_t s2 = nullptr;
  std::vector<hipEvent_t> ev;  // [0] fork, [1 + l] entropy of level l done
};
thread_local std::vector<Overlap> g_overlap;  // by device ordinal

hipError_t overlap_for(size_t n_levels, Overlap*& o) {
  int dev = 0;
  hipError_t r = hipGetDevice(&dev);
  if (r != hipSuccess) return r;
  if (g_overlap.size() <= (size_t)dev) g_overlap.resize(dev + 1);
  o = &g_overlap[dev];
  if (!o->s2) {
    r = hipStreamCreateWithFlags(&o->s2, hipStreamNonBlocking);
    if (r != hipSuccess) return r;
  }
  while (o->ev.size() < n_levels + 1) {
    hipEvent_t e = nullptr;
    r = hipEventCreateWithFlags(&e, hipEventDisableTiming);
    if (r != hipSuccess) return r;
    o->ev.push_back(e);
  }
  return hipSuccess;
}

// Launch-shape fields of a tuning record that the library offers.
int check_tuning(const ace_archive* A, const ace_tuning* t) {
  if (!t) return ACE_OK;
  const uint32_t w = t->waves_per_block, p = t->blocks_per_wg;
  if (w != 0 && w != 1 && w != 2 && w != 4 && w != 8)
    return fail(ACE_E_ARG, "waves_per_block %u: 1, 2, 4 or 8 (0 = by launch size)", w);
  if (p > 2 || (p == 2 && A->W > 32))
    return fail(ACE_E_ARG, "blocks_per_wg %u: 1, or 2 when the interleave is at most 32", p);
  if (t->lut_variant != 0) return fail(ACE_E_ARG, "lut_variant %u: only 0 is built", t->lut_variant);
  return ACE_OK;
}

// workspace header: error word (0), 16 counters of match bytes read from
// earlier blocks (16..144, one per block id mod 16)
constexpr uint64_t kWsHeader = 256, kWsCounters = 16;

uint32_t shift_of(uint32_t B) {
  if (B & (B - 1)) return 64;
  uint32_t k = 0;
  while ((1u << k) < B) k++;
  return k;
}

// Overlapped decode: levels [0, split) form the early group, whose entropy
// decode is one launch on the caller's stream; levels [split, n) are one
// launch on the second stream, running beside the early group's entropy
// decode and expansion.  The early group holds at most a quarter of the
// planned blocks (and at least level 0).
size_t level_split(const std::vector<uint32_t>& lstart) {
  const size_t nl = lstart.size() - 1;
  const uint64_t total = lstart[nl] - lstart[0];
  size_t split = 1;
  while (split + 1 < nl && 4ull * (lstart[split + 1] - lstart[0]) <= total) split++;
  return split;
}
constexpr uint32_t kModePersistent = 2, kModeOverlap = 3;  // 0 and 1: per level, one stream
// consecutive idle polls (each a sleep of about 1,000 cycles once idle for
// a while) before a persistent-kernel wait gives up and flags a timeout:
// about a second on this device
constexpr uint32_t kMaxIdlePolls = 1u << 21;

struct Layout {
  uint64_t plan, lv, loc, lit, lens, offs, slots, items, total;
};

// Workspace of one host-planned decode.  lv: per dependency level of the
// archive, the plan's level boundaries (depth + 1), then the persistent
// kernel's finished counts (depth) and its finished-level copies.
Layout layout(const ace_archive* A, uint64_t n_plan, uint64_t n_seq, uint64_t n_slots,
              uint64_t n_items) {
  Layout L;
  uint64_t o = kWsHeader;
  L.plan = o;  o = align_up(o + sizeof(PlanEntry) * n_plan, 256);
  L.lv = o;    o = align_up(o + 4ull * (persist_row(A->depth + 1) + persist_sync_words(A->depth)), 256);
  L.loc = o;   o = align_up(o + 8ull * A->nb, 256);
  L.lit = o;   o = align_up(o + (uint64_t)A->B * n_plan + 64, 256);  // +64: aligned over-read slack
  L.lens = o;  o = align_up(o + 4ull * n_seq, 256);
  L.offs = o;  o = align_up(o + (uint64_t)A->ow * n_seq, 256);
  L.slots = o; o = align_up(o + (uint64_t)A->B * n_slots, 256);
  L.items = o; o = align_up(o + sizeof(CopyItem) * n_items, 256);
  L.total = o;
  return L;
}

struct Plan {
  std::vector<PlanEntry> entries;  // level order
  std::vector<uint32_t> lstart;    // level boundaries in entries
  std::vector<CopyItem> items;
  uint64_t n_seq = 0;
  uint64_t n_slots = 0;
  bool use_slots_for_all = false;
};

// Marks the closure of the marked targets (dependencies are always earlier
// blocks, so one descending sweep from the highest target closes the set).
void close_set(const ace_archive* A, std::vector<uint8_t>& need, uint32_t top,
               std::vector<uint32_t>& blocks) {
  for (uint32_t b = top + 1; b-- > 0;) {
    if (!need[b]) continue;
    blocks.push_back(b);
    const BlockInfo& bi = A->blk[b];
    for (uint32_t j = 0; j < bi.dep_cnt; j++) need[A->deps[bi.dep_off + j]] = 1;
  }
}

// Closure of one range by a stack walk (touches only the closure).
void close_range(const ace_archive* A, uint32_t t0, uint32_t t1, std::vector<uint32_t>& blocks) {
  std::vector<uint32_t> stack;
  std::vector<uint8_t> seen(A->nb, 0);
  for (uint32_t b = t0; b <= t1; b++) {
    seen[b] = 1;
    stack.push_back(b);
  }
  while (!stack.empty()) {
    uint32_t b = stack.back();
    stack.pop_back();
    blocks.push_back(b);
    const BlockInfo& bi = A->blk[b];
    for (uint32_t j = 0; j < bi.dep_cnt; j++) {
      uint32_t d = A->deps[bi.dep_off + j];
      if (!seen[d]) {
        seen[d] = 1;
        stack.push_back(d);
      }
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// execution
// ---------------------------------------------------------------------------
static int run_launches(const ace_archive* A, const PlanEntry* entries, uint64_t n_plan,
                        const std::vector<uint32_t>& lstart, const CopyItem* items, uint64_t n_items,
                        const Layout& L, uint8_t* ws, uint64_t dst_base, const ace_tuning* t,
                        hipStream_t s, bool entries_pinned, bool loc_linear,
                        const PlanEntry* resident, const uint8_t* arch);

// Runs a host-built plan; with phase timing on, also records the host time
// spent planning (since the call's entry) and enqueueing.
static int run(const ace_archive* A, const PlanEntry* entries, uint64_t n_plan,
               const std::vector<uint32_t>& lstart, const CopyItem* items, uint64_t n_items,
               const Layout& L, uint8_t* ws, uint64_t dst_base, const ace_tuning* t,
               hipStream_t s, bool entries_pinned, bool loc_linear = false,
               const PlanEntry* resident = nullptr, const uint8_t* arch = nullptr) {
  if (!g_timer.on)
    return run_launches(A, entries, n_plan, lstart, items, n_items, L, ws, dst_base, t, s, entries_pinned,
                        loc_linear, resident, arch);
  const auto t_run = std::chrono::steady_clock::now();
  g_timer.us_plan = std::chrono::duration<double, std::micro>(t_run - g_timer.t_enter).count();
  const int rc = run_launches(A, entries, n_plan, lstart, items, n_items, L, ws, dst_base, t, s,
                              entries_pinned, loc_linear, resident, arch);
  g_timer.us_enqueue = us_since(t_run);
  return rc;
}

static int run_launches(const ace_archive* A, const PlanEntry* entries, uint64_t n_plan,
                        const std::vector<uint32_t>& lstart, const CopyItem* items, uint64_t n_items,
                        const Layout& L, uint8_t* ws, uint64_t dst_base, const ace_tuning* t,
                        hipStream_t s, bool entries_pinned, bool loc_linear,
                        const PlanEntry* resident, const uint8_t* arch) {
  (void)entries_pinned;
  if (!arch) arch = A->d_arch;  // an out-of-core seek passes its staged copy
  const uint32_t mode = t ? t->mode : 0;
  if (mode > 1 && mode != kModeOverlap && mode != kModePersistent) return fail(ACE_E_ARG, "unknown mode %u", mode);
  int rc = check_tuning(A, t);
  if (rc) return rc;
  const uint32_t waves = t ? t->waves_per_block : 0, per_wave = t ? t->blocks_per_wg : 0;
  DecodeArgs a{};
  a.arch = arch;
  a.plan = resident ? resident : reinterpret_cast<const PlanEntry*>(ws + L.plan);
  a.n_plan = (uint32_t)n_plan;
  a.B = A->B;
  a.b_shift = shift_of(A->B);
  a.W = A->W;
  a.ow = A->ow;
  a.n_blocks = A->nb;
  a.n_total = A->n;
  a.dst_base = dst_base;
  a.loc = reinterpret_cast<uint64_t*>(ws + L.loc);
  a.loc_linear = loc_linear ? 1u : 0u;
  a.lit = ws + L.lit;
  a.lens = ws + L.lens;
  a.offs = ws + L.offs;
  a.err = reinterpret_cast<uint32_t*>(ws);
  a.ext_bytes = reinterpret_cast<unsigned long long*>(ws + kWsCounters);
  a.n_lvl = (uint32_t)(lstart.size() - 1);
  a.lvl_dev = reinterpret_cast<const uint32_t*>(ws + L.lv);
  persist_sync(a, reinterpret_cast<uint32_t*>(ws + L.lv) + persist_row(a.n_lvl + 1));
  a.max_polls = kMaxIdlePolls;
  if (g_trace) {
    if (g_trace_entries < n_plan)
      return fail(ACE_E_NOSPACE, "the block trace holds %llu entries, the decode plans %llu",
                  (unsigned long long)g_trace_entries, (unsigned long long)n_plan);
    a.trace = g_trace;
  }
  if (n_plan && !resident) HIP_TRY(hipMemcpyAsync(ws + L.plan, entries, sizeof(PlanEntry) * n_plan,
                                     hipMemcpyHostToDevice, s));
  if (n_items) HIP_TRY(hipMemcpyAsync(ws + L.items, items, sizeof(CopyItem) * n_items,
                                      hipMemcpyHostToDevice, s));
  if (n_plan) {
    PhaseTimer& T = g_timer;
    const bool timed = T.on;
    T.n_ent = T.n_mat = 0;
    T.recorded = false;
    const size_t nl = lstart.size() - 1;
    auto expand = [&](size_t l) -> hipError_t {
      if (lstart[l + 1] <= lstart[l]) return hipSuccess;
      if (timed) {
        hipError_t r = timer_pair(T.mat, T.n_mat);
        if (r == hipSuccess) r = hipEventRecord(T.mat[2 * T.n_mat], s);
        if (r != hipSuccess) return r;
      }
      hipError_t r = launch_expand_level(a, lstart[l], lstart[l + 1], waves, s);
      if (r == hipSuccess && timed) r = hipEventRecord(T.mat[2 * T.n_mat++ + 1], s);
      return r;
    };
    auto entropy = [&](uint32_t lo, uint32_t hi, hipStream_t st) -> hipError_t {
      if (hi <= lo) return hipSuccess;
      if (timed) {
        hipError_t r = timer_pair(T.ent, T.n_ent);
        if (r == hipSuccess) r = hipEventRecord(T.ent[2 * T.n_ent], st);
        if (r != hipSuccess) return r;
      }
      hipError_t r = launch_rans(a, lo, hi, per_wave, st);
      if (r == hipSuccess && timed) r = hipEventRecord(T.ent[2 * T.n_ent++ + 1], st);
      return r;
    };
    if (mode == kModePersistent) {
      // the entropy launch, then one persistent launch for every level:
      // level boundaries uploaded, counters cleared by a fill kernel
      HIP_TRY(hipMemcpyAsync(ws + L.lv, lstart.data(), 4ull * lstart.size(), hipMemcpyHostToDevice, s));
      HIP_TRY(launch_fill_u32(a.lvl_done, 0u, persist_sync_words(a.n_lvl), s));
      HIP_TRY(entropy(0, (uint32_t)n_plan, s));
      if (timed) {
        HIP_TRY(timer_pair(T.mat, T.n_mat));
        HIP_TRY(hipEventRecord(T.mat[2 * T.n_mat], s));
      }
      HIP_TRY(launch_persistent(a, t ? t->grid_wgs : 0, s));
      if (timed) HIP_TRY(hipEventRecord(T.mat[2 * T.n_mat++ + 1], s));
    } else if (mode == kModeOverlap && nl > 1) {
      // fork: the late levels' entropy decode on the second stream; the
      // caller's stream decodes and expands the early levels meanwhile,
      // then waits for the late entropy decode and expands the rest
      const size_t split = level_split(lstart);
      Overlap* o = nullptr;
      HIP_TRY(overlap_for(1, o));
      HIP_TRY(hipEventRecord(o->ev[0], s));
      HIP_TRY(hipStreamWaitEvent(o->s2, o->ev[0], 0));
      HIP_TRY(entropy(lstart[split], lstart[nl], o->s2));
      HIP_TRY(hipEventRecord(o->ev[1], o->s2));
      HIP_TRY(entropy(lstart[0], lstart[split], s));
      for (size_t l = 0; l < split; l++) HIP_TRY(expand(l));
      HIP_TRY(hipStreamWaitEvent(s, o->ev[1], 0));
      for (size_t l = split; l < nl; l++) HIP_TRY(expand(l));
    } else {
      HIP_TRY(entropy(0, (uint32_t)n_plan, s));
      for (size_t l = 0; l < nl; l++) HIP_TRY(expand(l));
    }
    T.recorded = timed;
  }
  if (n_items)
    HIP_TRY(launch_copy(a, reinterpret_cast<const CopyItem*>(ws + L.items), (uint32_t)n_items, s));
  return ACE_OK;
}

extern "C" int ace_workspace_bytes(const ace_archive* A, const ace_range* r, uint32_t n,
                                   uint64_t* bytes) {
  if (!A || !bytes || (n && !r)) return fail(ACE_E_ARG, "null argument");
  if (n == 0) {
    *bytes = layout(A, A->nb, A->all_seq, 0, 0).total;
    return ACE_OK;
  }
  std::vector<uint8_t> need(A->nb, 0);
  uint32_t top = 0;
  uint64_t items = 0;
  bool any = false;
  for (uint32_t i = 0; i < n; i++) {
    if (r[i].lo > r[i].hi) return fail(ACE_E_ARG, "range %u is inverted", i);
    if (r[i].hi > A->n) return fail(ACE_E_RANGE, "range %u ends beyond %llu", i, (unsigned long long)A->n);
    if (r[i].lo == r[i].hi) continue;
    uint32_t t0 = (uint32_t)(r[i].lo / A->B), t1 = (uint32_t)((r[i].hi - 1) / A->B);
    for (uint32_t b = t0; b <= t1; b++) need[b] = 1;
    top = std::max(top, t1);
    items += (r[i].hi - r[i].lo + 65535) / 65536 + 2;
    any = true;
  }
  std::vector<uint32_t> blocks;
  if (any) close_set(A, need, top, blocks);
  uint64_t seq = 0;
  for (uint32_t b : blocks) seq += A->blk[b].n_seq;
  *bytes = layout(A, blocks.size(), seq, blocks.size(), items).total;
  return ACE_OK;
}

extern "C" int ace_decode_all(const ace_archive* A, uint8_t* d_out, uint64_t out_cap, void* d_ws,
                              uint64_t ws_cap, const ace_tuning* t, void* stream) {
  timer_enter();
  if (!A || (!d_out && A->n) || !d_ws) return fail(ACE_E_ARG, "null argument");
  if (int rc = need_resident(A)) return rc;
  if (out_cap < A->n) return fail(ACE_E_NOSPACE, "output needs %llu bytes", (unsigned long long)A->n);
  Layout L = layout(A, A->nb, A->all_seq, 0, 0);
  if (ws_cap < L.total) return fail(ACE_E_NOSPACE, "workspace needs %llu bytes", (unsigned long long)L.total);
  if (A->nb == 0) return ACE_OK;
  if (A->d_plan)
    return run(A, A->all_plan.data(), A->nb, A->all_levels, nullptr, 0, L, static_cast<uint8_t*>(d_ws),
               (uint64_t)(uintptr_t)d_out, t, static_cast<hipStream_t>(stream), false, true, A->d_plan);
  ace_archive* M = const_cast<ace_archive*>(A);
  const PlanEntry* entries = A->all_plan.data();
  {
    std::lock_guard<std::mutex> g(M->pin_mu);
    if (!M->all_plan_pinned) {
      void* p = nullptr;
      if (hipHostMalloc(&p, sizeof(PlanEntry) * A->nb, hipHostMallocDefault) == hipSuccess) {
        memcpy(p, A->all_plan.data(), sizeof(PlanEntry) * A->nb);
        M->all_plan_pinned = static_cast<PlanEntry*>(p);
      } else {
        (void)hipGetLastError();
      }
    }
    if (M->all_plan_pinned) entries = M->all_plan_pinned;
  }
  return run(A, entries, A->nb, A->all_levels, nullptr, 0, L, static_cast<uint8_t*>(d_ws),
             (uint64_t)(uintptr_t)d_out, t, static_cast<hipStream_t>(stream), true, true);
}

// The resident plan: the entries, then the blocks by level and the level
// boundaries (the static data of device-side seek planning).
static uint64_t plan_bytes(const ace_archive* A) {
  return sizeof(PlanEntry) * (uint64_t)A->nb + 4ull * A->nb + 4ull * (A->depth + 1);
}

extern "C" int ace_plan_bytes(const ace_archive* A, uint64_t* bytes) {
  if (!A || !bytes) return fail(ACE_E_ARG, "null argument");
  *bytes = plan_bytes(A);
  return ACE_OK;
}

extern "C" int ace_archive_attach_plan(ace_archive* A, void* d_plan, uint64_t bytes, void* stream) {
  if (!A || (!d_plan && A->nb)) return fail(ACE_E_ARG, "null argument");
  if (int rc = need_resident(A)) return rc;
  const uint64_t need = plan_bytes(A);
  if (bytes < need) return fail(ACE_E_NOSPACE, "the plan needs %llu bytes", (unsigned long long)need);
  if (A->nb == 0) return ACE_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<uint32_t> order(A->nb);
  for (uint32_t i = 0; i < A->nb; i++) order[i] = A->all_plan[i].block;
  uint8_t* d = static_cast<uint8_t*>(d_plan);
  const uint64_t o_order = sizeof(PlanEntry) * (uint64_t)A->nb, o_lstart = o_order + 4ull * A->nb;
  HIP_TRY(hipMemcpyAsync(d, A->all_plan.data(), o_order, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d + o_order, order.data(), 4ull * A->nb, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d + o_lstart, A->all_levels.data(), 4ull * (A->depth + 1), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  A->d_plan = reinterpret_cast<const PlanEntry*>(d);
  A->d_order = reinterpret_cast<const uint32_t*>(d + o_order);
  A->d_lstart = reinterpret_cast<const uint32_t*>(d + o_lstart);
  return ACE_OK;
}

static uint64_t seek_device_bytes(const ace_archive* A);
static int seek_device(const ace_archive* A, uint64_t lo, uint64_t hi, uint8_t* d_out, uint8_t* ws,
                       const ace_tuning* t, hipStream_t s);

// One seek into the workspace ws (whole target blocks straight into d_out
// on the host-planned path).  Planned on the device when the archive's plan
// is resident and ws holds seek_device_bytes (allow_device), else the
// closure of [lo, hi) is planned on the host.  ws_need, when given, receives
// the workspace size the host-planned seek needs (also on ACE_E_NOSPACE).
static int seek_impl(const ace_archive* A, uint64_t lo, uint64_t hi, uint8_t* d_out, void* d_ws,
                     uint64_t ws_cap, const ace_tuning* t, void* stream, uint64_t* ws_need,
                     bool allow_device = true) {
  timer_enter();
  if (!A) return fail(ACE_E_ARG, "null archive");
  if (int rc = need_resident(A)) return rc;
  if (lo > hi) return fail(ACE_E_ARG, "inverted range [%llu, %llu)", (unsigned long long)lo,
                           (unsigned long long)hi);
  if (hi > A->n) return fail(ACE_E_RANGE, "range end %llu beyond %llu", (unsigned long long)hi,
                             (unsigned long long)A->n);
  if (lo == hi) return ACE_OK;
  if (!d_out || !d_ws) return fail(ACE_E_ARG, "null argument");
  if (allow_device && A->d_order && ws_cap >= seek_device_bytes(A)) {
    if (ws_need) *ws_need = seek_device_bytes(A);
    return seek_device(A, lo, hi, d_out, static_cast<uint8_t*>(d_ws), t, static_cast<hipStream_t>(stream));
  }
  const uint32_t t0 = (uint32_t)(lo / A->B), t1 = (uint32_t)((hi - 1) / A->B);
  std::vector<uint32_t> blocks, order, lstart;
  close_range(A, t0, t1, blocks);
  level_order(A, blocks, order, lstart);
  // locations: whole target blocks go straight to the output
  std::vector<PlanEntry> entries(order.size());
  std::vector<CopyItem> items;
  uint64_t seq = 0, n_slots = 0;
  std::vector<uint8_t> direct(order.size(), 0);
  for (size_t i = 0; i < order.size(); i++) {
    const uint32_t b = order[i];
    const uint64_t bs = (uint64_t)b * A->B, be = std::min<uint64_t>(bs + A->B, A->n);
    direct[i] = b >= t0 && b <= t1 && bs >= lo && be <= hi;
    if (!direct[i]) n_slots++;
    entries[i] = make_entry(A, b, seq, 0);
    seq += A->blk[b].n_seq;
  }
  for (uint32_t b : {t0, t1}) {
    const uint64_t bs = (uint64_t)b * A->B, be = std::min<uint64_t>(bs + A->B, A->n);
    if (bs >= lo && be <= hi) continue;
    if (b == t1 && t1 == t0 && !items.empty()) continue;
    const uint64_t s0 = std::max(lo, bs), s1 = std::min(hi, be);
    items.push_back(CopyItem{s0, (uint64_t)(uintptr_t)d_out + (s0 - lo), (uint32_t)(s1 - s0), 0});
  }
  Layout L = layout(A, order.size(), seq, n_slots, items.size());
  if (ws_need) *ws_need = L.total;
  if (ws_cap < L.total) return fail(ACE_E_NOSPACE, "workspace needs %llu bytes", (unsigned long long)L.total);
  uint8_t* ws = static_cast<uint8_t*>(d_ws);
  uint64_t slot = 0;
  for (size_t i = 0; i < order.size(); i++) {
    const uint64_t bs = (uint64_t)order[i] * A->B;
    entries[i].dst = direct[i] ? (uint64_t)(uintptr_t)d_out + (bs - lo)
                               : (uint64_t)(uintptr_t)(ws + L.slots) + (slot++) * A->B;
  }
  return run(A, entries.data(), entries.size(), lstart, items.data(), items.size(), L, ws, 0, t,
             static_cast<hipStream_t>(stream), false);
}

extern "C" int ace_seek(const ace_archive* A, uint64_t lo, uint64_t hi, uint8_t* d_out, void* d_ws,
                        uint64_t ws_cap, const ace_tuning* t, void* stream) {
  return seek_impl(A, lo, hi, d_out, d_ws, ws_cap, t, stream, nullptr);
}

// ---------------------------------------------------------------------------
// out-of-core range decode
// ---------------------------------------------------------------------------
// An out-of-core seek is the host-planned seek with the archive bytes it
// reads staged into its workspace: the dependency lists of the planned
// blocks, then their payloads (each 16-aligned, ACE_ARCH_PAD readable bytes
// after the last).  The kernels address the archive as base + offset (the
// dependency array at the index's place, kHdr + 32 * n_blocks, payloads at
// their offsets), so the plan entries get offsets into the staged copy and
// the base is placed kHdr + 32 * n_blocks before it; the staged copy starts
// at least that far into the workspace, so the base stays inside it.
namespace {
struct OocSeek {
  std::vector<uint32_t> order, lstart;
  std::vector<PlanEntry> entries;
  std::vector<CopyItem> items;
  std::vector<uint8_t> direct;
  uint64_t seq = 0, n_slots = 0, deps_bytes = 0, pay_bytes = 0;
  Layout L{};
  uint64_t gap = 0, stage = 0, total = 0;
};

void ooc_plan(const ace_archive* A, uint64_t lo, uint64_t hi, uint8_t* d_out, OocSeek& P) {
  const uint32_t t0 = (uint32_t)(lo / A->B), t1 = (uint32_t)((hi - 1) / A->B);
  std::vector<uint32_t> blocks;
  close_range(A, t0, t1, blocks);
  level_order(A, blocks, P.order, P.lstart);
  P.entries.resize(P.order.size());
  P.direct.assign(P.order.size(), 0);
  for (size_t i = 0; i < P.order.size(); i++) {
    const uint32_t b = P.order[i];
    const uint64_t bs = (uint64_t)b * A->B, be = std::min<uint64_t>(bs + A->B, A->n);
    P.direct[i] = b >= t0 && b <= t1 && bs >= lo && be <= hi;
    if (!P.direct[i]) P.n_slots++;
    P.entries[i] = make_entry(A, b, P.seq, 0);
    P.seq += A->blk[b].n_seq;
    P.deps_bytes += 4ull * A->blk[b].dep_cnt;
    P.pay_bytes += align_up(A->blk[b].plen, 16);
  }
  for (uint32_t b : {t0, t1}) {
    const uint64_t bs = (uint64_t)b * A->B, be = std::min<uint64_t>(bs + A->B, A->n);
    if (bs >= lo && be <= hi) continue;
    if (b == t1 && t1 == t0 && !P.items.empty()) continue;
    const uint64_t s0 = std::max(lo, bs), s1 = std::min(hi, be);
    P.items.push_back(CopyItem{s0, (uint64_t)(uintptr_t)d_out + (s0 - lo), (uint32_t)(s1 - s0), 0});
  }
  P.L = layout(A, P.order.size(), P.seq, P.n_slots, P.items.size());
  P.gap = kHdr + (uint64_t)kBlk * A->nb;
  P.stage = align_up(std::max(P.L.total, P.gap), 256);
  P.total = P.stage + align_up(P.deps_bytes, 16) + P.pay_bytes + ACE_ARCH_PAD;
}
}  // namespace

extern "C" int ace_seek_ooc_bytes(const ace_archive* A, uint64_t lo, uint64_t hi, uint64_t* bytes) {
  if (!A || !bytes) return fail(ACE_E_ARG, "null argument");
  if (lo > hi) return fail(ACE_E_ARG, "inverted range [%llu, %llu)", (unsigned long long)lo,
                           (unsigned long long)hi);
  if (hi > A->n) return fail(ACE_E_RANGE, "range end %llu beyond %llu", (unsigned long long)hi,
                             (unsigned long long)A->n);
  if (lo == hi) {
    *bytes = 0;
    return ACE_OK;
  }
  OocSeek P;
  ooc_plan(A, lo, hi, nullptr, P);
  *bytes = P.total;
  return ACE_OK;
}

extern "C" int ace_seek_ooc(const ace_archive* A, uint64_t lo, uint64_t hi, uint8_t* d_out, void* d_ws,
                            uint64_t ws_cap, const ace_tuning* t, void* stream) {
  timer_enter();
  if (!A) return fail(ACE_E_ARG, "null archive");
  if (!A->h_arch) return fail(ACE_E_ARG, "the archive was not opened out of core (ace_archive_open_ooc)");
  if (lo > hi) return fail(ACE_E_ARG, "inverted range [%llu, %llu)", (unsigned long long)lo,
                           (unsigned long long)hi);
  if (hi > A->n) return fail(ACE_E_RANGE, "range end %llu beyond %llu", (unsigned long long)hi,
                             (unsigned long long)A->n);
  if (lo == hi) return ACE_OK;
  if (!d_out || !d_ws) return fail(ACE_E_ARG, "null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  OocSeek P;
  ooc_plan(A, lo, hi, d_out, P);
  if (ws_cap < P.total) return fail(ACE_E_NOSPACE, "workspace needs %llu bytes", (unsigned long long)P.total);
  uint8_t* ws = static_cast<uint8_t*>(d_ws);
  uint64_t slot = 0;
  for (size_t i = 0; i < P.order.size(); i++) {
    const uint64_t bs = (uint64_t)P.order[i] * A->B;
    P.entries[i].dst = P.direct[i] ? (uint64_t)(uintptr_t)d_out + (bs - lo)
                                   : (uint64_t)(uintptr_t)(ws + P.L.slots) + (slot++) * A->B;
  }
  // one staging buffer per archive: calls on it take turns, each finished
  // on its stream before the next one refills the buffer
  ace_archive* M = const_cast<ace_archive*>(A);
  std::lock_guard<std::mutex> g(M->ooc_mu);
  const uint64_t staged = align_up(P.deps_bytes, 16) + P.pay_bytes;
  if (M->ooc_pinned_cap < staged) {
    if (M->ooc_pinned) (void)hipHostFree(M->ooc_pinned);
    M->ooc_pinned = nullptr;
    M->ooc_pinned_cap = 0;
    void* p = nullptr;
    HIP_TRY(hipHostMalloc(&p, staged, hipHostMallocDefault));
    M->ooc_pinned = static_cast<uint8_t*>(p);
    M->ooc_pinned_cap = staged;
  }
  uint8_t* h = M->ooc_pinned;
  // the dependency lists, then the payloads; each 4 MiB packed is copied
  // while the host packs the next (the copies are asynchronous from pinned
  // memory, and each reads only bytes already packed)
  uint64_t dpos = 0;
  for (PlanEntry& e : P.entries) {
    const BlockInfo& bi = A->blk[e.block];
    memcpy(h + dpos, A->deps.data() + bi.dep_off, 4ull * bi.dep_cnt);
    e.dep_off = (uint32_t)(dpos / 4);
    dpos += 4ull * bi.dep_cnt;
  }
  constexpr uint64_t kChunk = 4ull << 20;
  uint64_t sent = 0, ppos = align_up(P.deps_bytes, 16);
  for (PlanEntry& e : P.entries) {
    const BlockInfo& bi = A->blk[e.block];
    memcpy(h + ppos, A->h_arch + bi.pay, bi.plen);
    const uint64_t pay = P.gap + ppos;  // offset from the kernels' archive base
    for (int k = 0; k < 3; k++)
      if (e.raw[k] != kCoded) e.raw[k] = e.raw[k] - bi.pay + pay;
    e.pay = pay;
    ppos += align_up(bi.plen, 16);
    if (ppos - sent >= kChunk) {
      HIP_TRY(hipMemcpyAsync(ws + P.stage + sent, h + sent, ppos - sent, hipMemcpyHostToDevice, s));
      sent = ppos;
    }
  }
  if (staged > sent) HIP_TRY(hipMemcpyAsync(ws + P.stage + sent, h + sent, staged - sent, hipMemcpyHostToDevice, s));
  const int rc = run(A, P.entries.data(), P.entries.size(), P.lstart, P.items.data(), P.items.size(), P.L, ws, 0,
                     t, s, false, false, nullptr, ws + P.stage - P.gap);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(s));
  return ACE_OK;
}

static_assert(kStaticScratchBytes == ACE_STATIC_SCRATCH_BYTES, "the fixed scratch size the header states");

extern "C" int ace_seek_static(const ace_archive* A, uint64_t lo, uint64_t hi, uint8_t* d_out,
                               uint32_t* d_status, const ace_tuning* t, void* stream) {
  if (!A || !d_status) return fail(ACE_E_ARG, "null argument");
  if (t && t->mode != 0 && t->mode != 1)
    return fail(ACE_E_ARG, "the allocation-free seek runs the per-level path (mode 0 or 1), not mode %u", t->mode);
  if (g_timer.on) return fail(ACE_E_ARG, "phase timing creates events; turn it off for the allocation-free seek");
  hipStream_t s = static_cast<hipStream_t>(stream);
  void* ws = nullptr;
  HIP_TRY(static_scratch(&ws));
  // the error word and the counters start at zero (a fill kernel: no memset
  // node if the caller captures this call)
  HIP_TRY(launch_fill_u32(static_cast<uint32_t*>(ws), 0u, kWsHeader / 4, s));
  uint64_t need = 0;
  int rc = seek_impl(A, lo, hi, d_out, ws, kStaticScratchBytes, t, stream, &need, false);
  if (rc == ACE_E_NOSPACE)
    return fail(ACE_E_NOSPACE, "the seek needs %llu bytes of scratch; the fixed scratch holds %llu",
                (unsigned long long)need, (unsigned long long)kStaticScratchBytes);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(d_status, ws, 4, hipMemcpyDeviceToDevice, s));
  return ACE_OK;
}

extern "C" int ace_seek_batch(const ace_archive* A, const ace_range* r, uint32_t n, uint8_t* d_out,
                              const uint64_t* out_off, void* d_ws, uint64_t ws_cap,
                              const ace_tuning* t, void* stream) {
  timer_enter();
  if (!A || (n && (!r || !out_off))) return fail(ACE_E_ARG, "null argument");
  if (int rc = need_resident(A)) return rc;
  std::vector<uint8_t> need(A->nb, 0);
  uint32_t top = 0;
  bool any = false;
  std::vector<CopyItem> items;
  for (uint32_t i = 0; i < n; i++) {
    if (r[i].lo > r[i].hi) return fail(ACE_E_ARG, "range %u is inverted", i);
    if (r[i].hi > A->n) return fail(ACE_E_RANGE, "range %u ends beyond %llu", i, (unsigned long long)A->n);
    if (r[i].lo == r[i].hi) continue;
    if (!d_out || !d_ws) return fail(ACE_E_ARG, "null argument");
    const uint32_t t0 = (uint32_t)(r[i].lo / A->B), t1 = (uint32_t)((r[i].hi - 1) / A->B);
    for (uint32_t b = t0; b <= t1; b++) need[b] = 1;
    top = std::max(top, t1);
    any = true;
    for (uint64_t s0 = r[i].lo; s0 < r[i].hi; s0 += 65536) {
      const uint64_t s1 = std::min<uint64_t>(s0 + 65536, r[i].hi);
      items.push_back(CopyItem{s0, (uint64_t)(uintptr_t)d_out + out_off[i] + (s0 - r[i].lo),
                               (uint32_t)(s1 - s0), 0});
    }
  }
  if (!any) return ACE_OK;
  std::vector<uint32_t> blocks, order, lstart;
  close_set(A, need, top, blocks);
  level_order(A, blocks, order, lstart);
  uint64_t seq = 0;
  for (uint32_t b : order) seq += A->blk[b].n_seq;
  Layout L = layout(A, order.size(), seq, order.size(), items.size());
  if (ws_cap < L.total) return fail(ACE_E_NOSPACE, "workspace needs %llu bytes", (unsigned long long)L.total);
  uint8_t* ws = static_cast<uint8_t*>(d_ws);
  std::vector<PlanEntry> entries(order.size());
  uint64_t sq = 0;
  for (size_t i = 0; i < order.size(); i++) {
    entries[i] = make_entry(A, order[i], sq, (uint64_t)(uintptr_t)(ws + L.slots) + i * (uint64_t)A->B);
    sq += A->blk[order[i]].n_seq;
  }
  return run(A, entries.data(), entries.size(), lstart, items.data(), items.size(), L, ws, 0, t,
             static_cast<hipStream_t>(stream), false);
}

extern "C" int ace_check(void* d_ws, void* stream) {
  if (!d_ws) return fail(ACE_E_ARG, "null workspace");
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipStreamSynchronize(s));
  uint32_t err = 0, zero = 0;
  HIP_TRY(hipMemcpy(&err, d_ws, 4, hipMemcpyDeviceToHost));
  if (err) HIP_TRY(hipMemcpy(d_ws, &zero, 4, hipMemcpyHostToDevice));
  if (err & kErrTimeout) return fail(ACE_E_TIMEOUT, "a dependency wait on the device expired");
  if (err & kErrCorrupt) return fail(ACE_E_CORRUPT, "a token stream broke a format rule");
  return ACE_OK;
}

extern "C" int ace_read_counters(void* d_ws, void* stream, uint64_t* ext_src_bytes) {
  if (!d_ws || !ext_src_bytes) return fail(ACE_E_ARG, "null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipStreamSynchronize(s));
  uint64_t v[16] = {0}, zero[16] = {0};
  HIP_TRY(hipMemcpy(v, static_cast<uint8_t*>(d_ws) + kWsCounters, sizeof(v), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(static_cast<uint8_t*>(d_ws) + kWsCounters, zero, sizeof(zero), hipMemcpyHostToDevice));
  uint64_t sum = 0;
  for (uint64_t c : v) sum += c;
  *ext_src_bytes = sum;
  return ACE_OK;
}

// ---------------------------------------------------------------------------
// Batched seek as one replayed HIP graph (device-side planning).
// ---------------------------------------------------------------------------
struct ace_batch {
  const ace_archive* A = nullptr;
  uint32_t cap = 0;
  hipStream_t stream = nullptr;
  uint8_t* ws = nullptr;
  uint64_t off_desc = 0;
  uint64_t* staging = nullptr;  // pinned host copy of the descriptors
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  bool pending = false;
  hipStream_t s2 = nullptr;     // the entropy branch of the captured graph
  std::vector<hipEvent_t> ev;   // fork + one per level (capture edges only)
  DecodeArgs a{};               // the captured decode's arguments
  uint32_t waves = 0, per_wave = 0;
  uint64_t off_plan = 0, off_pin = 0, off_pinbase = 0;
  uint32_t pinned_levels = 0;
};

namespace {
struct BatchLayout {
  uint64_t order, lstart, need, pre, plan, nplan, lvl, loc, lit, lens, offs, slots, desc, pin, pinbase,
      chunks, total;
};

BatchLayout batch_layout(const ace_archive* A, uint32_t cap) {
  BatchLayout L;
  uint64_t o = kWsHeader;
  auto take = [&](uint64_t bytes) {
    uint64_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.order = take(4ull * A->nb);
  L.lstart = take(4ull * (A->depth + 1));
  L.need = take(align_up(A->nb, 4));
  L.pre = take(4ull * A->nb);
  L.plan = take(sizeof(PlanEntry) * A->nb);
  L.nplan = take(4);
  L.lvl = take(4ull * (persist_row(A->depth + 1) + persist_sync_words(A->depth)));  // plan boundaries, then the persistent kernel's counters
  L.loc = take(8ull * A->nb);
  L.lit = take((uint64_t)A->B * A->nb + 64);
  L.lens = take(4ull * A->all_seq);
  L.offs = take((uint64_t)A->ow * A->all_seq);
  L.slots = take((uint64_t)A->B * A->nb);
  L.desc = take(16 + 24ull * cap);
  L.pin = take(align_up(A->nb, 4));
  L.pinbase = take(4);
  L.chunks = take(8ull * (batch_compact_chunks(A->nb) + 1));
  L.total = o;
  return L;
}
}  // namespace

static uint64_t seek_device_bytes(const ace_archive* A) { return batch_layout(A, 1).total; }

// A device-planned seek: the batch planner for one request (mark the target
// blocks, close level by level, compact into a level-ordered plan), the
// device-planned decode into workspace slots, then the copy of [lo, hi) to
// d_out.  The host only enqueues: no closure walk.  The static planning data
// (blocks by level, level boundaries) come from the resident plan.
static int seek_device(const ace_archive* A, uint64_t lo, uint64_t hi, uint8_t* d_out, uint8_t* ws,
                       const ace_tuning* t, hipStream_t s) {
  const uint32_t mode = t ? t->mode : 0;
  if (mode > 1 && mode != kModeOverlap && mode != kModePersistent) return fail(ACE_E_ARG, "unknown mode %u", mode);
  int rc = check_tuning(A, t);
  if (rc) return rc;
  const BatchLayout L = batch_layout(A, 1);
  BatchArgs ba{};
  ba.arch = A->d_arch;
  ba.B = A->B;
  ba.n_blocks = A->nb;
  ba.depth = A->depth;
  ba.cap = 1;
  ba.n_total = A->n;
  ba.order = A->d_order;
  ba.lstart = A->d_lstart;
  ba.need = ws + L.need;
  ba.pre = reinterpret_cast<uint32_t*>(ws + L.pre);
  ba.desc = reinterpret_cast<const uint64_t*>(ws + L.desc);
  ba.plan = reinterpret_cast<PlanEntry*>(ws + L.plan);
  ba.n_plan_dev = reinterpret_cast<uint32_t*>(ws + L.nplan);
  ba.lvl_dev = reinterpret_cast<uint32_t*>(ws + L.lvl);
  ba.loc = reinterpret_cast<uint64_t*>(ws + L.loc);
  ba.pin = ws + L.pin;
  ba.pin_base = reinterpret_cast<const uint32_t*>(ws + L.pinbase);
  ba.chunk_cnt = reinterpret_cast<uint32_t*>(ws + L.chunks);
  ba.chunk_seq = ba.chunk_cnt + batch_compact_chunks(A->nb) + 1;
  DecodeArgs a{};
  a.arch = A->d_arch;
  a.plan = ba.plan;
  a.n_plan = A->nb;  // capacity: the real count is read on the device
  a.B = A->B;
  a.b_shift = shift_of(A->B);
  a.W = A->W;
  a.ow = A->ow;
  a.n_blocks = A->nb;
  a.n_total = A->n;
  a.dst_base = (uint64_t)(uintptr_t)(ws + L.slots);
  a.loc = ba.loc;
  a.lit = ws + L.lit;
  a.lens = ws + L.lens;
  a.offs = ws + L.offs;
  a.err = reinterpret_cast<uint32_t*>(ws);
  a.ext_bytes = reinterpret_cast<unsigned long long*>(ws + kWsCounters);
  a.n_plan_dev = ba.n_plan_dev;
  a.lvl_dev = ba.lvl_dev;
  a.n_lvl = A->depth;
  persist_sync(a, ba.lvl_dev + persist_row(A->depth + 1));
  a.max_polls = kMaxIdlePolls;
  if (g_trace) {
    if (g_trace_entries < A->nb)
      return fail(ACE_E_NOSPACE, "the block trace holds %llu entries, a device-planned seek may plan %u",
                  (unsigned long long)g_trace_entries, A->nb);
    a.trace = g_trace;
  }
  const uint32_t waves = t ? t->waves_per_block : 0, per_wave = t ? t->blocks_per_wg : 0;
  PhaseTimer& T = g_timer;
  const bool timed = T.on;
  std::chrono::steady_clock::time_point t_run;
  if (timed) {
    t_run = std::chrono::steady_clock::now();
    T.us_plan = std::chrono::duration<double, std::micro>(t_run - T.t_enter).count();
    T.n_ent = T.n_mat = 0;
    T.recorded = false;
    HIP_TRY(timer_pair(T.ent, 0));
    HIP_TRY(timer_pair(T.mat, 0));
  }
  // request descriptor, marks and the (empty) kept-block table (the header's
  // error word and counters accumulate as for every other call)
  HIP_TRY(launch_put_range(reinterpret_cast<uint64_t*>(ws + L.desc), (uint64_t)(uintptr_t)d_out, lo, hi, s));
  HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(ws + L.need), 0u, align_up(A->nb, 4) / 4, s));
  HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(ws + L.pin), 0u, align_up(A->nb, 4) / 4, s));
  HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(ws + L.pinbase), 0u, 1, s));
  HIP_TRY(launch_batch_mark(ba, s));
  for (uint32_t l = A->depth; l-- > 1;)
    HIP_TRY(launch_batch_close(ba, l, A->all_levels[l + 1] - A->all_levels[l], s));
  HIP_TRY(launch_batch_compact(ba, s));
  if (timed) HIP_TRY(hipEventRecord(T.ent[0], s));
  if (mode == kModePersistent) {
    HIP_TRY(launch_fill_u32(a.lvl_done, 0u, persist_sync_words(A->depth), s));
    HIP_TRY(launch_rans_dev(a, A->nb, per_wave, s));
    if (timed) {
      HIP_TRY(hipEventRecord(T.ent[1], s));
      HIP_TRY(hipEventRecord(T.mat[0], s));
    }
    HIP_TRY(launch_persistent(a, t ? t->grid_wgs : 0, s));
  } else {
    // modes 0, 1 and 3: one entropy launch, then one expansion per level
    HIP_TRY(launch_rans_dev(a, A->nb, per_wave, s));
    if (timed) {
      HIP_TRY(hipEventRecord(T.ent[1], s));
      HIP_TRY(hipEventRecord(T.mat[0], s));
    }
    for (uint32_t l = 0; l < A->depth; l++)
      HIP_TRY(launch_expand_level_dev(a, l, A->all_levels[l + 1] - A->all_levels[l], waves, s));
  }
  if (timed) HIP_TRY(hipEventRecord(T.mat[1], s));
  HIP_TRY(launch_batch_gather(ba, a, s));
  if (timed) {
    T.n_ent = T.n_mat = 1;
    T.recorded = true;
    T.us_enqueue = us_since(t_run);
  }
  return ACE_OK;
}

extern "C" int ace_workspace_bound(const ace_archive* A, uint32_t n_ranges, uint64_t total_bytes,
                                   uint64_t* bytes) {
  if (!A || !bytes) return fail(ACE_E_ARG, "null argument");
  // every block planned, every one in a slot, and the most copy items the
  // ranges can need: a range of len bytes takes at most len / 64 KiB + 3
  // (the layout grows with each of these)
  const uint64_t items = total_bytes / 65536 + 3ull * n_ranges;
  *bytes = layout(A, A->nb, A->all_seq, A->nb, items).total;
  return ACE_OK;
}

extern "C" int ace_batch_workspace_bytes(const ace_archive* A, uint32_t max_requests,
                                         uint64_t* bytes) {
  if (!A || !bytes) return fail(ACE_E_ARG, "null argument");
  *bytes = batch_layout(A, max_requests).total;
  return ACE_OK;
}

extern "C" void ace_batch_destroy(ace_batch* b) {
  if (!b) return;
  if (b->pending) (void)hipEventSynchronize(b->done);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->done) (void)hipEventDestroy(b->done);
  for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
  if (b->s2) (void)hipStreamDestroy(b->s2);
  if (b->staging) (void)hipHostFree(b->staging);
  delete b;
}

extern "C" int ace_batch_create(const ace_archive* A, uint32_t cap, void* d_ws, uint64_t ws_cap,
                                const ace_tuning* t, void* stream, ace_batch** out) {
  if (!A || !d_ws || !out || cap == 0) return fail(ACE_E_ARG, "null argument or zero capacity");
  if (int rc = need_resident(A)) return rc;
  if (!stream) return fail(ACE_E_ARG, "a batch needs a stream of its own: the default stream cannot be captured");
  const BatchLayout L = batch_layout(A, cap);
  if (ws_cap < L.total) return fail(ACE_E_NOSPACE, "workspace needs %llu bytes", (unsigned long long)L.total);
  ace_batch* b = new (std::nothrow) ace_batch();
  if (!b) return fail(ACE_E_NOMEM, "out of memory");
  b->A = A;
  b->cap = cap;
  b->stream = static_cast<hipStream_t>(stream);
  b->ws = static_cast<uint8_t*>(d_ws);
  b->off_desc = L.desc;
  hipStream_t s = b->stream;
  int rc = ACE_OK;
  do {
    if (hipHostMalloc((void**)&b->staging, 16 + 24ull * cap, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) {
      rc = fail(ACE_E_HIP, "pinned staging or event allocation failed");
      break;
    }
    // static planning data: all blocks by level, and the level boundaries
    std::vector<uint32_t> order(A->nb);
    for (uint32_t i = 0; i < A->nb; i++) order[i] = A->all_plan[i].block;
    uint32_t widest = 0;
    for (uint32_t l = 0; l < A->depth; l++)
      widest = std::max(widest, A->all_levels[l + 1] - A->all_levels[l]);
    if (hipMemcpyAsync(b->ws + L.order, order.data(), 4ull * A->nb, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(b->ws + L.lstart, A->all_levels.data(), 4ull * (A->depth + 1),
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = fail(ACE_E_HIP, "upload of the level order failed");
      break;
    }
    BatchArgs ba{};
    ba.arch = A->d_arch;
    ba.B = A->B;
    ba.n_blocks = A->nb;
    ba.depth = A->depth;
    ba.cap = cap;
    ba.n_total = A->n;
    ba.order = reinterpret_cast<const uint32_t*>(b->ws + L.order);
    ba.lstart = reinterpret_cast<const uint32_t*>(b->ws + L.lstart);
    ba.need = b->ws + L.need;
    ba.pre = reinterpret_cast<uint32_t*>(b->ws + L.pre);
    ba.desc = reinterpret_cast<const uint64_t*>(b->ws + L.desc);
    ba.plan = reinterpret_cast<PlanEntry*>(b->ws + L.plan);
    ba.n_plan_dev = reinterpret_cast<uint32_t*>(b->ws + L.nplan);
    ba.lvl_dev = reinterpret_cast<uint32_t*>(b->ws + L.lvl);
    ba.loc = reinterpret_cast<uint64_t*>(b->ws + L.loc);
    ba.pin = b->ws + L.pin;
    ba.pin_base = reinterpret_cast<const uint32_t*>(b->ws + L.pinbase);
    ba.chunk_cnt = reinterpret_cast<uint32_t*>(b->ws + L.chunks);
    ba.chunk_seq = ba.chunk_cnt + batch_compact_chunks(A->nb) + 1;
    b->off_plan = L.plan;
    b->off_pin = L.pin;
    b->off_pinbase = L.pinbase;
    // nothing kept yet: every block is planned when needed, from slot 0
    if (launch_fill_u32(reinterpret_cast<uint32_t*>(b->ws + L.pin), 0u, align_up(A->nb, 4) / 4, s) != hipSuccess ||
        launch_fill_u32(reinterpret_cast<uint32_t*>(b->ws + L.pinbase), 0u, 1, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = fail(ACE_E_HIP, "clearing the kept-block table failed");
      break;
    }
    DecodeArgs a{};
    a.arch = A->d_arch;
    a.plan = ba.plan;
    a.n_plan = A->nb;  // capacity: the real count is read on the device
    a.B = A->B;
    a.b_shift = shift_of(A->B);
    a.W = A->W;
    a.ow = A->ow;
    a.n_blocks = A->nb;
    a.n_total = A->n;
    a.dst_base = (uint64_t)(uintptr_t)(b->ws + L.slots);
    a.loc = ba.loc;
    a.lit = b->ws + L.lit;
    a.lens = b->ws + L.lens;
    a.offs = b->ws + L.offs;
    a.err = reinterpret_cast<uint32_t*>(b->ws);
    a.ext_bytes = reinterpret_cast<unsigned long long*>(b->ws + kWsCounters);
    a.n_plan_dev = ba.n_plan_dev;
    a.lvl_dev = ba.lvl_dev;
    a.n_lvl = A->depth;
    persist_sync(a, ba.lvl_dev + persist_row(A->depth + 1));
    a.max_polls = kMaxIdlePolls;
    const uint32_t mode = t ? t->mode : 0;
    if (mode > 1 && mode != kModeOverlap && mode != kModePersistent) {
      rc = fail(ACE_E_ARG, "unknown mode %u", mode);
      break;
    }
    if ((rc = check_tuning(A, t)) != ACE_OK) break;
    const uint32_t waves = t ? t->waves_per_block : 0, per_wave = t ? t->blocks_per_wg : 0;
    b->a = a;
    b->waves = waves;
    b->per_wave = per_wave;
    // the late levels' entropy decode on a branch of the graph, beside the
    // early levels' decode (mode 3)
    const bool overlap = mode == kModeOverlap && A->depth > 1;
    if (overlap) {
      bool ok = hipStreamCreateWithFlags(&b->s2, hipStreamNonBlocking) == hipSuccess;
      for (uint32_t l = 0; ok && l < 2; l++) {
        hipEvent_t ev = nullptr;
        ok = hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
        if (ok) b->ev.push_back(ev);
      }
      if (!ok) {
        rc = fail(ACE_E_HIP, "stream or event creation failed");
        break;
      }
    }
    if (waves == 0 && prepare_expand_shapes() != hipSuccess) {
      rc = fail(ACE_E_HIP, "device occupancy query failed");
      break;
    }
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      rc = fail(ACE_E_HIP, "graph capture could not start");
      break;
    }
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(ba.need), 0u, align_up(A->nb, 4) / 4, s);
    if (e == hipSuccess) e = launch_batch_mark(ba, s);
    for (uint32_t l = A->depth; e == hipSuccess && l-- > 1;)
      e = launch_batch_close(ba, l, A->all_levels[l + 1] - A->all_levels[l], s);
    if (e == hipSuccess) e = launch_batch_compact(ba, s);
    if (e == hipSuccess && mode == kModePersistent) {
      e = launch_fill_u32(a.lvl_done, 0u, persist_sync_words(A->depth), s);
      if (e == hipSuccess) e = launch_rans_dev(a, A->nb, per_wave, s);
      if (e == hipSuccess) e = launch_persistent(a, t ? t->grid_wgs : 0, s);
    } else if (e == hipSuccess && overlap) {
      const size_t split = level_split(A->all_levels);
      const uint32_t nl = A->depth;
      e = hipEventRecord(b->ev[0], s);
      if (e == hipSuccess) e = hipStreamWaitEvent(b->s2, b->ev[0], 0);
      if (e == hipSuccess)
        e = launch_rans_levels_dev(a, (uint32_t)split, nl, A->all_levels[nl] - A->all_levels[split], per_wave,
                                   b->s2);
      if (e == hipSuccess) e = hipEventRecord(b->ev[1], b->s2);
      if (e == hipSuccess)
        e = launch_rans_levels_dev(a, 0, (uint32_t)split, A->all_levels[split] - A->all_levels[0], per_wave, s);
      for (uint32_t l = 0; e == hipSuccess && l < nl; l++) {
        if (l == split) e = hipStreamWaitEvent(s, b->ev[1], 0);
        if (e == hipSuccess)
          e = launch_expand_level_dev(a, l, A->all_levels[l + 1] - A->all_levels[l], waves, s);
      }
    } else if (e == hipSuccess) {
      e = launch_rans_dev(a, A->nb, per_wave, s);
      for (uint32_t l = 0; e == hipSuccess && l < A->depth; l++)
        e = launch_expand_level_dev(a, l, A->all_levels[l + 1] - A->all_levels[l], waves, s);
    }
    if (e == hipSuccess) e = launch_batch_gather(ba, a, s);
    hipError_t e2 = hipStreamEndCapture(s, &b->graph);
    if (e != hipSuccess || e2 != hipSuccess) {
      rc = fail(ACE_E_HIP, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
      break;
    }
    if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
      rc = fail(ACE_E_HIP, "graph instantiation failed");
      break;
    }
    (void)widest;
  } while (0);
  if (rc) {
    ace_batch_destroy(b);
    return rc;
  }
  *out = b;
  return ACE_OK;
}

extern "C" int ace_batch_pin(ace_batch* b, uint32_t levels) {
  if (!b) return fail(ACE_E_ARG, "null argument");
  const ace_archive* A = b->A;
  if (b->pinned_levels) return fail(ACE_E_ARG, "this batch already keeps %u levels", b->pinned_levels);
  if (levels > A->depth) return fail(ACE_E_ARG, "%u levels requested, the archive has %u", levels, A->depth);
  if (levels == 0) return ACE_OK;
  // the plan, token scratch and slots are shared with the replays
  if (b->pending) HIP_TRY(hipEventSynchronize(b->done));
  b->pending = false;
  hipStream_t s = b->stream;
  // levels [0, levels) are a prefix of the whole-archive level order and are
  // closed under dependencies: entry i decodes into slot i
  const uint32_t P = A->all_levels[levels];
  std::vector<PlanEntry> e(A->all_plan.begin(), A->all_plan.begin() + P);
  for (uint32_t i = 0; i < P; i++) e[i].dst = (uint64_t)i * A->B;
  std::vector<uint8_t> pin(align_up(A->nb, 4), 0);
  for (uint32_t i = 0; i < P; i++) pin[e[i].block] = 1;
  DecodeArgs a = b->a;
  a.plan = reinterpret_cast<const PlanEntry*>(b->ws + b->off_plan);
  a.n_plan = P;
  a.n_plan_dev = nullptr;
  a.lvl_dev = nullptr;
  HIP_TRY(hipMemcpyAsync(b->ws + b->off_plan, e.data(), sizeof(PlanEntry) * P, hipMemcpyHostToDevice, s));
  HIP_TRY(launch_rans(a, 0, P, b->per_wave, s));
  for (uint32_t l = 0; l < levels; l++)
    HIP_TRY(launch_expand_level(a, A->all_levels[l], A->all_levels[l + 1], b->waves, s));
  HIP_TRY(hipStreamSynchronize(s));
  uint32_t err = 0;
  HIP_TRY(hipMemcpy(&err, b->ws, 4, hipMemcpyDeviceToHost));
  if (err) {  // reported here, so cleared; nothing is marked kept
    const uint32_t zero = 0;
    HIP_TRY(hipMemcpy(b->ws, &zero, 4, hipMemcpyHostToDevice));
    return fail(ACE_E_CORRUPT, "decoding the kept levels failed (device error word 0x%x)", err);
  }
  // only a complete decode is marked kept
  HIP_TRY(hipMemcpyAsync(b->ws + b->off_pin, pin.data(), pin.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(b->ws + b->off_pinbase, &P, 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  b->pinned_levels = levels;
  return ACE_OK;
}

extern "C" int ace_batch_run(ace_batch* b, const ace_range* r, uint32_t n, uint8_t* d_out,
                             const uint64_t* out_off) {
  if (!b || (n && (!r || !out_off || !d_out))) return fail(ACE_E_ARG, "null argument");
  if (n > b->cap) return fail(ACE_E_ARG, "%u requests exceed the batch capacity %u", n, b->cap);
  for (uint32_t i = 0; i < n; i++) {
    if (r[i].lo > r[i].hi) return fail(ACE_E_ARG, "range %u is inverted", i);
    if (r[i].hi > b->A->n) return fail(ACE_E_RANGE, "range %u ends beyond %llu", i, (unsigned long long)b->A->n);
  }
  // the staging buffer is reused: the previous replay must have read it
  if (b->pending) HIP_TRY(hipEventSynchronize(b->done));
  b->staging[0] = n;
  b->staging[1] = (uint64_t)(uintptr_t)d_out;
  for (uint32_t i = 0; i < n; i++) {
    b->staging[2 + 3 * i] = r[i].lo;
    b->staging[3 + 3 * i] = r[i].hi;
    b->staging[4 + 3 * i] = out_off[i];
  }
  HIP_TRY(hipMemcpyAsync(b->ws + b->off_desc, b->staging, 16 + 24ull * n, hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipGraphLaunch(b->exec, b->stream));
  HIP_TRY(hipEventRecord(b->done, b->stream));
  b->pending = true;
  return ACE_OK;
}

extern "C" int ace_set_block_trace(void* d_trace, uint64_t bytes) {
  if (d_trace && bytes < 64) return fail(ACE_E_NOSPACE, "a block trace needs 64 bytes per planned block");
  g_trace = static_cast<unsigned long long*>(d_trace);
  g_trace_entries = d_trace ? bytes / 64 : 0;
  return ACE_OK;
}

extern "C" int ace_set_timing(int on) {
  g_timer.on = on != 0;
  g_timer.recorded = false;
  return ACE_OK;
}

extern "C" int ace_last_timings(float* ms_entropy, float* ms_match) {
  if (!ms_entropy || !ms_match) return fail(ACE_E_ARG, "null argument");
  const PhaseTimer& T = g_timer;
  if (!T.recorded) return fail(ACE_E_ARG, "no timed decode on this thread");
  float e = 0, m = 0;
  for (size_t k = 0; k < T.n_ent; k++) {
    float t = 0;
    HIP_TRY(hipEventSynchronize(T.ent[2 * k + 1]));
    HIP_TRY(hipEventElapsedTime(&t, T.ent[2 * k], T.ent[2 * k + 1]));
    e += t;
  }
  for (size_t k = 0; k < T.n_mat; k++) {
    float t = 0;
    HIP_TRY(hipEventSynchronize(T.mat[2 * k + 1]));
    HIP_TRY(hipEventElapsedTime(&t, T.mat[2 * k], T.mat[2 * k + 1]));
    m += t;
  }
  *ms_entropy = e;
  *ms_match = m;
  return ACE_OK;
}

extern "C" int ace_last_host_times(double* us_plan, double* us_enqueue) {
  if (!us_plan || !us_enqueue) return fail(ACE_E_ARG, "null argument");
  if (!g_timer.recorded) return fail(ACE_E_ARG, "no timed decode on this thread");
  *us_plan = g_timer.us_plan;
  *us_enqueue = g_timer.us_enqueue;
  return ACE_OK;
}
