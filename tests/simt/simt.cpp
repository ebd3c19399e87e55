// Host implementation of the HIP stand-in declared in hip/hip_runtime.h: a
// fiber-per-lane wavefront scheduler and a synchronous runtime.  Test
// infrastructure only.
#include "hip/hip_runtime.h"

#include <sched.h>
#include <stdio.h>
#include <stdlib.h>
#include <sys/mman.h>
#include <ucontext.h>

#include <chrono>
#include <mutex>
#include <thread>
#include <vector>

namespace simt {
namespace {

enum St { kRun, kWaveWait, kBarWait, kDone };
enum Op { kBallot, kReadlane, kReadfirst, kDpp, kShfl, kShflXor, kWaveBar, kBar, kBarOr };

struct Lane {
  ucontext_t ctx;
  uint32_t tid = 0;
  int st = kRun;
  int op = 0;
  uint32_t v = 0, a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  uint64_t res = 0;
};

struct Wg {
  std::vector<Lane> lanes;
  uint32_t n = 0;
  uint3 bid{0, 0, 0}, bdim{1, 1, 1}, gdim{1, 1, 1};
  ucontext_t sched;
  const std::function<void()>* body = nullptr;
};

thread_local Wg* t_wg = nullptr;
thread_local Lane* t_lane = nullptr;
thread_local std::vector<void*> t_stacks;

constexpr size_t kStack = 256 << 10;

[[noreturn]] void fatal(const char* what) {
  fprintf(stderr, "simt: %s (block %u,%u lane %u)\n", what, t_wg ? t_wg->bid.x : 0u, t_wg ? t_wg->bid.y : 0u,
          t_lane ? t_lane->tid : 0u);
  fflush(stderr);
  abort();
}

void lane_main() {
  (*t_wg->body)();
  t_lane->st = kDone;
  swapcontext(&t_lane->ctx, &t_wg->sched);
  fatal("a finished lane was resumed");
}

uint64_t collective(int op, uint32_t v, uint32_t a0 = 0, uint32_t a1 = 0, uint32_t a2 = 0, uint32_t a3 = 0) {
  if (!t_lane) fatal("cross-lane operation outside a kernel");
  Lane* l = t_lane;
  l->op = op;
  l->v = v;
  l->a0 = a0;
  l->a1 = a1;
  l->a2 = a2;
  l->a3 = a3;
  l->st = (op == kBar || op == kBarOr) ? kBarWait : kWaveWait;
  swapcontext(&l->ctx, &t_wg->sched);
  return t_lane->res;
}

uint32_t dpp_one(const Lane* const* w, uint32_t l, uint32_t old, int ctl, int row_mask, bool bound_ctrl) {
  const uint32_t row = l / 16, pos = l % 16;
  if (!((row_mask >> row) & 1)) return old;
  int src = -1;
  if (ctl >= 0x111 && ctl <= 0x11F) {
    const uint32_t k = (uint32_t)ctl - 0x110;
    if (pos >= k) src = (int)(l - k);
  } else if (ctl >= 0 && ctl <= 0xFF) {  // quad_perm: lane q of each quad reads lane (ctl >> 2q) & 3
    src = (int)((l & ~3u) + (((uint32_t)ctl >> (2 * (l & 3))) & 3u));
  } else if (ctl == 0x142) {  // row_bcast:15
    if (row > 0) src = (int)(16 * (row - 1) + 15);
  } else if (ctl == 0x143) {  // row_bcast:31
    if (row >= 2) src = 31;
  } else {
    fatal("DPP control not modelled");
  }
  if (src < 0 || !w[src]) return bound_ctrl ? 0u : old;
  return w[src]->v;
}

void resolve_wave(Lane* const* w) {
  int op = -1;
  uint32_t a0 = 0, a1 = 0;
  for (uint32_t l = 0; l < 64; l++) {
    if (!w[l]) continue;
    if (op < 0) {
      op = w[l]->op;
      a0 = w[l]->a0;
      a1 = w[l]->a1;
    } else if (w[l]->op != op) {
      fatal("lanes of one wave reached different cross-lane operations");
    } else if ((op == kReadlane || op == kDpp) && (w[l]->a0 != a0 || w[l]->a1 != a1)) {
      fatal("non-uniform operand of a uniform cross-lane operation");
    }
  }
  switch (op) {
    case kBallot: {
      uint64_t m = 0;
      for (uint32_t l = 0; l < 64; l++)
        if (w[l] && w[l]->v) m |= 1ull << l;
      for (uint32_t l = 0; l < 64; l++)
        if (w[l]) w[l]->res = m;
      break;
    }
    case kReadlane: {
      if (a0 >= 64 || !w[a0]) fatal("readlane of a lane that is not live");
      for (uint32_t l = 0; l < 64; l++)
        if (w[l]) w[l]->res = w[a0]->v;
      break;
    }
    case kReadfirst: {
      uint32_t first = 64;
      for (uint32_t l = 0; l < 64 && first == 64; l++)
        if (w[l]) first = l;
      for (uint32_t l = 0; l < 64; l++)
        if (w[l]) w[l]->res = w[first]->v;
      break;
    }
    case kDpp: {
      uint64_t out[64];
      for (uint32_t l = 0; l < 64; l++)
        if (w[l]) {
          if (w[l]->a2 != 0xF) fatal("DPP bank mask not modelled");
          out[l] = dpp_one(w, l, w[l]->a3, (int)w[l]->a0, (int)w[l]->a1, false);
        }
      for (uint32_t l = 0; l < 64; l++)
        if (w[l]) w[l]->res = out[l];
      break;
    }
    case kShfl:
    case kShflXor: {
      uint64_t out[64];
      for (uint32_t l = 0; l < 64; l++) {
        if (!w[l]) continue;
        const uint32_t width = w[l]->a1 ? w[l]->a1 : 64;
        const uint32_t seg = l & ~(width - 1);
        const uint32_t src = op == kShfl ? seg + (w[l]->a0 & (width - 1)) : (l ^ w[l]->a0);
        if (src >= 64 || !w[src]) fatal("shuffle from a lane that is not live");
        out[l] = w[src]->v;
      }
      for (uint32_t l = 0; l < 64; l++)
        if (w[l]) w[l]->res = out[l];
      break;
    }
    case kWaveBar:
      break;
    default:
      fatal("unknown cross-lane operation");
  }
  for (uint32_t l = 0; l < 64; l++)
    if (w[l]) w[l]->st = kRun;
}

void run_wg(Wg& g) {
  const uint32_t n = g.n;
  while (t_stacks.size() < n) {
    void* p = mmap(nullptr, kStack, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
    if (p == MAP_FAILED) fatal("no memory for lane stacks");
    t_stacks.push_back(p);
  }
  g.lanes.assign(n, Lane());
  t_wg = &g;
  for (uint32_t i = 0; i < n; i++) {
    Lane& l = g.lanes[i];
    l.tid = i;
    l.st = kRun;
    getcontext(&l.ctx);
    l.ctx.uc_stack.ss_sp = t_stacks[i];
    l.ctx.uc_stack.ss_size = kStack;
    l.ctx.uc_link = nullptr;
    makecontext(&l.ctx, (void (*)())lane_main, 0);
  }
  const uint32_t nw = (n + 63) / 64;
  for (;;) {
    for (uint32_t i = 0; i < n; i++) {
      if (g.lanes[i].st != kRun) continue;
      t_lane = &g.lanes[i];
      swapcontext(&g.sched, &g.lanes[i].ctx);
    }
    t_lane = nullptr;
    bool moved = false;
    for (uint32_t w = 0; w < nw; w++) {
      Lane* ln[64] = {};
      uint32_t live = 0, wave_wait = 0, bar_wait = 0;
      for (uint32_t l = 0; l < 64 && 64 * w + l < n; l++) {
        Lane& x = g.lanes[64 * w + l];
        if (x.st == kDone) continue;
        ln[l] = &x;
        live++;
        if (x.st == kWaveWait) wave_wait++;
        if (x.st == kBarWait) bar_wait++;
      }
      if (!live || !wave_wait) continue;
      if (bar_wait) fatal("lanes of one wave split between a barrier and a cross-lane operation");
      resolve_wave(ln);
      moved = true;
    }
    if (moved) continue;
    uint32_t live = 0, bar = 0;
    bool any = false;
    int op = -1;
    for (uint32_t i = 0; i < n; i++) {
      Lane& x = g.lanes[i];
      if (x.st == kDone) continue;
      live++;
      if (x.st == kBarWait) {
        bar++;
        any = any || x.v;
        if (op < 0) op = x.op;
        else if (op != x.op) fatal("lanes reached different barriers");
      }
    }
    if (!live) break;
    if (bar != live) fatal("workgroup deadlock");
    for (uint32_t i = 0; i < n; i++) {
      Lane& x = g.lanes[i];
      if (x.st == kDone) continue;
      x.res = any ? 1 : 0;
      x.st = kRun;
    }
  }
  t_wg = nullptr;
}

uint32_t resident() {
  static uint32_t r = [] {
    const char* e = getenv("SIMT_RESIDENT");
    int v = e ? atoi(e) : 8;
    return (uint32_t)(v > 0 ? v : 8);
  }();
  return r;
}

thread_local hipError_t t_err = hipSuccess;

}  // namespace

uint3 thread_idx() {
  const uint32_t t = t_lane->tid, bx = t_wg->bdim.x, by = t_wg->bdim.y;
  return uint3{t % bx, (t / bx) % by, t / (bx * by)};
}
uint3 block_idx() { return t_wg->bid; }
uint3 block_dim() { return t_wg->bdim; }
uint3 grid_dim() { return t_wg->gdim; }
uint32_t lane_id() { return t_lane->tid & 63; }

uint64_t ballot(bool p) { return collective(kBallot, p ? 1u : 0u); }
uint32_t readlane(uint32_t v, uint32_t lane) { return (uint32_t)collective(kReadlane, v, lane); }
uint32_t readfirstlane(uint32_t v) { return (uint32_t)collective(kReadfirst, v); }
uint32_t dpp(uint32_t old, uint32_t src, int ctl, int row_mask, int bank_mask, bool bound_ctrl) {
  if (bound_ctrl) fatal("DPP bound_ctrl not modelled");
  return (uint32_t)collective(kDpp, src, (uint32_t)ctl, (uint32_t)row_mask, (uint32_t)bank_mask, old);
}
uint32_t shfl(uint32_t v, int src, int width) { return (uint32_t)collective(kShfl, v, (uint32_t)src, (uint32_t)width); }
uint32_t shfl_xor(uint32_t v, int mask, int width) {
  return (uint32_t)collective(kShflXor, v, (uint32_t)mask, (uint32_t)width);
}
void wave_barrier() { collective(kWaveBar, 0); }
void syncthreads() { collective(kBar, 0); }
bool syncthreads_or(bool p) { return collective(kBarOr, p ? 1u : 0u) != 0; }
void spin_pause() { sched_yield(); }
uint64_t steady_ticks() {
  using namespace std::chrono;
  return (uint64_t)duration_cast<nanoseconds>(steady_clock::now().time_since_epoch()).count() / 1000;  // a 1 MHz clock: host emulation runs far slower than the GPU
}

}  // namespace simt

// ---------------------------------------------------------------------------
// runtime
// ---------------------------------------------------------------------------
struct ihipStream_t {
  bool capturing = false;
  std::vector<std::function<void()>> ops;
};
struct ihipEvent_t {
  std::chrono::steady_clock::time_point t;
};
struct ihipGraph_t {
  std::vector<std::function<void()>> ops;
};
struct ihipGraphExec_t {
  std::vector<std::function<void()>> ops;
};

namespace simt {
namespace {
void launch_now(dim3 g, dim3 b, const std::function<void()>& body) {
  const uint64_t total = (uint64_t)g.x * g.y * g.z;
  if (!total) return;
  const uint32_t nthr = (uint32_t)(total < resident() ? total : resident());
  std::atomic<uint64_t> next{0};
  auto worker = [&]() {
    for (;;) {
      const uint64_t i = next.fetch_add(1);
      if (i >= total) break;
      Wg w;
      w.n = b.x * b.y * b.z;
      w.bdim = uint3{b.x, b.y, b.z};
      w.gdim = uint3{g.x, g.y, g.z};
      w.bid = uint3{(uint32_t)(i % g.x), (uint32_t)((i / g.x) % g.y), (uint32_t)(i / ((uint64_t)g.x * g.y))};
      w.body = &body;
      run_wg(w);
    }
  };
  std::vector<std::thread> th;
  for (uint32_t k = 0; k < nthr; k++) th.emplace_back(worker);
  for (auto& t : th) t.join();
}
}  // namespace

void launch(dim3 g, dim3 b, hipStream_t s, std::function<void()> body) {
  if (s && s->capturing) {
    s->ops.push_back([g, b, body]() { launch_now(g, b, body); });
    return;
  }
  launch_now(g, b, body);
}
}  // namespace simt

hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int) {
  *v = a == hipDeviceAttributeMultiprocessorCount ? (int)simt::resident() : 0;
  return hipSuccess;
}
hipError_t hipGetLastError() {
  hipError_t e = simt::t_err;
  simt::t_err = hipSuccess;
  return e;
}
hipError_t hipPeekAtLastError() { return simt::t_err; }
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "simulated error"; }

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t s) {
  if (s && s->capturing) {
    s->ops.push_back([dst, src, n]() { memcpy(dst, src, n); });
    return hipSuccess;
  }
  if (n) memcpy(dst, src, n);
  return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind k) {
  return hipMemcpyAsync(dst, src, n, k, nullptr);
}
hipError_t hipMemsetAsync(void* dst, int v, size_t n, hipStream_t s) {
  if (s && s->capturing) {
    s->ops.push_back([dst, v, n]() { memset(dst, v, n); });
    return hipSuccess;
  }
  memset(dst, v, n);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned) {
  *p = malloc(n ? n : 1);
  return *p ? hipSuccess : hipErrorUnknown;
}
hipError_t hipHostFree(void* p) {
  free(p);
  return hipSuccess;
}
hipError_t hipMalloc(void** p, size_t n) { return hipHostMalloc(p, n, 0); }
hipError_t hipFree(void* p) { return hipHostFree(p); }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = new ihipStream_t();
  return hipSuccess;
}
hipError_t hipStreamCreate(hipStream_t* s) { return hipStreamCreateWithFlags(s, 0); }
hipError_t hipStreamDestroy(hipStream_t s) {
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new ihipEvent_t();
  (*e)->t = std::chrono::steady_clock::now();
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  if (s && s->capturing) {
    s->ops.push_back([e]() { e->t = std::chrono::steady_clock::now(); });
    return hipSuccess;
  }
  e->t = std::chrono::steady_clock::now();
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  *ms = std::chrono::duration<float, std::milli>(b->t - a->t).count();
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  if (!s || s->capturing) return hipErrorInvalidValue;
  s->capturing = true;
  s->ops.clear();
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  if (!s || !s->capturing) return hipErrorInvalidValue;
  s->capturing = false;
  *g = new ihipGraph_t();
  (*g)->ops.swap(s->ops);
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  *x = new ihipGraphExec_t();
  (*x)->ops = g->ops;
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
  if (s && s->capturing) {
    s->ops.push_back([x]() {
      for (auto& f : x->ops) f();
    });
    return hipSuccess;
  }
  for (auto& f : x->ops) f();
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
  delete x;
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete g;
  return hipSuccess;
}

// A stream for callers of the CPU build that need one of their own (graph
// capture refuses the null stream).
extern "C" void* simt_stream_create() {
  hipStream_t s = nullptr;
  hipStreamCreate(&s);
  return s;
}
