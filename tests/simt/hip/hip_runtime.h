// Host stand-in for the HIP runtime header, used only to build the library's
// kernel and host sources as ordinary x86 C++ for CPU checks (test
// infrastructure; the product is always built with hipcc for gfx950).
//
// Execution model: a workgroup runs on one OS thread; each of its lanes is a
// cooperative fiber.  Lanes run one after another between cross-lane points
// (ballot, DPP, shuffles, readlane, wave and workgroup barriers), where the
// scheduler waits for every live lane of the wave (or workgroup) and then
// computes the results as a 64-wide wavefront would.  A cross-lane operation
// must therefore be reached by every live lane of the wave, which the
// kernels' own contracts already require.  LDS (__shared__) is one object per
// OS thread, so workgroups that run at the same time have their own, and a
// thread's later workgroups see what the earlier ones left (as LDS does).
// Up to `resident` workgroups of a launch run at once, taken in block order,
// so kernels that wait on each other see the residency they were sized for.
#pragma once
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <atomic>
#include <functional>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline __attribute__((always_inline))
#define __launch_bounds__(...)
#define __shared__ static thread_local
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(x) ((const void*)&(x))
// occupancy hints name GPU register budgets; on the host they mean nothing
#define amdgpu_waves_per_eu(...) unused

struct uint3 {
  uint32_t x, y, z;
};
struct dim3 {
  uint32_t x, y, z;
  constexpr dim3(uint32_t a = 1, uint32_t b = 1, uint32_t c = 1) : x(a), y(b), z(c) {}
};
struct uint4 {
  uint32_t x, y, z, w;
};
inline uint4 make_uint4(uint32_t a, uint32_t b, uint32_t c, uint32_t d) { return uint4{a, b, c, d}; }

typedef int hipError_t;
enum : int {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorNotSupported = 801,
  hipErrorUnknown = 999,
};
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost,
                     hipMemcpyDeviceToDevice, hipMemcpyDefault };
enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount = 1, hipDeviceAttributeOther = 2 };
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal, hipStreamCaptureModeThreadLocal,
                            hipStreamCaptureModeRelaxed };
constexpr unsigned hipStreamNonBlocking = 1, hipEventDisableTiming = 2, hipHostMallocDefault = 0;

struct ihipStream_t;
struct ihipEvent_t;
struct ihipGraph_t;
struct ihipGraphExec_t;
typedef ihipStream_t* hipStream_t;
typedef ihipEvent_t* hipEvent_t;
typedef ihipGraph_t* hipGraph_t;
typedef ihipGraphExec_t* hipGraphExec_t;
typedef ihipGraph_t* hipGraphNode_t;

namespace simt {

uint3 thread_idx();
uint3 block_idx();
uint3 block_dim();
uint3 grid_dim();

// cross-lane operations (every live lane of the wave takes part)
uint64_t ballot(bool p);
uint32_t readlane(uint32_t v, uint32_t lane);
uint32_t readfirstlane(uint32_t v);
uint32_t dpp(uint32_t old, uint32_t src, int ctl, int row_mask, int bank_mask, bool bound_ctrl);
uint32_t shfl(uint32_t v, int src, int width);
uint32_t shfl_xor(uint32_t v, int mask, int width);
void wave_barrier();
void syncthreads();
bool syncthreads_or(bool p);
uint32_t lane_id();
void spin_pause();
uint64_t steady_ticks();

void launch(dim3 grid, dim3 block, hipStream_t s, std::function<void()> body);

}  // namespace simt

#define threadIdx (::simt::thread_idx())
#define blockIdx (::simt::block_idx())
#define blockDim (::simt::block_dim())
#define gridDim (::simt::grid_dim())

#define hipLaunchKernelGGL(kernel, grid, block, shmem, stream, ...) \
  ::simt::launch(dim3(grid), dim3(block), (stream), [=]() { kernel(__VA_ARGS__); })

// wave builtins
#define __builtin_amdgcn_update_dpp(old, src, ctl, rm, bm, bc) \
  ((int)::simt::dpp((uint32_t)(old), (uint32_t)(src), (ctl), (rm), (bm), (bc)))
#define __builtin_amdgcn_ballot_w64(p) ::simt::ballot(p)
#define __builtin_amdgcn_readlane(v, l) ((int)::simt::readlane((uint32_t)(v), (uint32_t)(l)))
#define __builtin_amdgcn_readfirstlane(v) ((int)::simt::readfirstlane((uint32_t)(v)))
#define __builtin_amdgcn_s_sleep(n) ::simt::spin_pause()
#define __builtin_amdgcn_fence(order, ...) std::atomic_thread_fence(std::memory_order_seq_cst)
#define __builtin_amdgcn_s_barrier() ::simt::syncthreads()
#define __builtin_amdgcn_wave_barrier() ::simt::wave_barrier()
#define __builtin_amdgcn_rcpf(x) (1.0f / (float)(x))
// v_perm_b32: byte i of the result is byte sel_i of src0:src1 (src1 the low
// dword); selectors 0..7 pick bytes, 12 gives 0x00, 13 gives 0xFF
inline uint32_t simt_perm(uint32_t src0, uint32_t src1, uint32_t sel) {
  const uint64_t v = ((uint64_t)src0 << 32) | src1;
  uint32_t r = 0;
  for (uint32_t i = 0; i < 4; i++) {
    const uint32_t k = (sel >> (8 * i)) & 0xFFu;
    const uint32_t b = k < 8 ? (uint32_t)(v >> (8 * k)) & 0xFFu : k == 13 ? 0xFFu : 0u;
    r |= b << (8 * i);
  }
  return r;
}
#define __builtin_amdgcn_perm(src0, src1, sel) simt_perm((uint32_t)(src0), (uint32_t)(src1), (uint32_t)(sel))
#define __builtin_amdgcn_alignbyte(hi, lo, k) \
  ((uint32_t)(((((uint64_t)(uint32_t)(hi)) << 32) | (uint32_t)(lo)) >> (8 * ((uint32_t)(k) & 3u))))

inline uint32_t __builtin_amdgcn_mbcnt_lo(uint32_t m, uint32_t base) {
  const uint32_t l = ::simt::lane_id();
  const uint32_t below = l >= 32 ? 0xFFFFFFFFu : ((1u << l) - 1u);
  return base + (uint32_t)__builtin_popcount(m & below);
}
inline uint32_t __builtin_amdgcn_mbcnt_hi(uint32_t m, uint32_t base) {
  const uint32_t l = ::simt::lane_id();
  const uint32_t below = l < 32 ? 0u : ((1u << (l - 32)) - 1u);
  return base + (uint32_t)__builtin_popcount(m & below);
}

inline uint64_t __ballot(bool p) { return ::simt::ballot(p); }
template <typename T>
inline T __shfl(T v, int src, int width = 64) {
  return (T)::simt::shfl((uint32_t)v, src, width);
}
template <typename T>
inline T __shfl_xor(T v, int mask, int width = 64) {
  return (T)::simt::shfl_xor((uint32_t)v, mask, width);
}
template <typename T>
inline T __shfl_up(T v, unsigned d, int width = 64) {
  const int l = (int)::simt::lane_id();
  const int src = (l % width) >= (int)d ? l - (int)d : l;
  return (T)::simt::shfl((uint32_t)v, src % width, width);
}
inline void __syncthreads() { ::simt::syncthreads(); }
inline int __syncthreads_or(int p) { return ::simt::syncthreads_or(p != 0) ? 1 : 0; }
inline void __threadfence() { std::atomic_thread_fence(std::memory_order_seq_cst); }

template <typename T>
inline T max(T a, T b) { return a > b ? a : b; }
template <typename T>
inline T min(T a, T b) { return a < b ? a : b; }
inline int __popc(uint32_t v) { return __builtin_popcount(v); }
inline int __popcll(uint64_t v) { return __builtin_popcountll(v); }
inline int __clz(uint32_t v) { return v ? __builtin_clz(v) : 32; }
inline int __ffs(uint32_t v) { return __builtin_ffs(v); }
inline uint32_t __umul24(uint32_t a, uint32_t b) { return (a & 0xFFFFFFu) * (b & 0xFFFFFFu); }
inline long long wall_clock64() { return (long long)::simt::steady_ticks(); }

#define __HIP_MEMORY_SCOPE_WAVEFRONT 2
#define __HIP_MEMORY_SCOPE_WORKGROUP 3
#define __HIP_MEMORY_SCOPE_AGENT 4
#define __HIP_MEMORY_SCOPE_SYSTEM 5

// __hip_atomic_* are clang builtins on the host as well.
template <typename T>
inline T __simt_fetch_max(T* p, T v) {
  T cur = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while (cur < v && !__atomic_compare_exchange_n(p, &cur, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
  }
  return cur;
}

template <typename T, typename U>
inline T atomicAdd(T* p, U v) {
  return __atomic_fetch_add(p, (T)v, __ATOMIC_SEQ_CST);
}
template <typename T, typename U>
inline T atomicSub(T* p, U v) {
  return __atomic_fetch_sub(p, (T)v, __ATOMIC_SEQ_CST);
}
template <typename T, typename U>
inline T atomicOr(T* p, U v) {
  return __atomic_fetch_or(p, (T)v, __ATOMIC_SEQ_CST);
}
template <typename T, typename U>
inline T atomicMax(T* p, U v) {
  return __simt_fetch_max(p, (T)v);
}
template <typename T, typename U>
inline T atomicExch(T* p, U v) {
  return __atomic_exchange_n(p, (T)v, __ATOMIC_SEQ_CST);
}
template <typename T, typename U, typename V>
inline T atomicCAS(T* p, U expected, V desired) {
  T e = (T)expected;
  __atomic_compare_exchange_n(p, &e, (T)desired, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST);
  return e;  // the value found (equal to expected when the exchange happened)
}
// s_getreg: the XCC_ID register (20) reads as the workgroup index mod 8,
// the round-robin placement of workgroups over eight XCDs; other
// registers read as 0
inline uint32_t simt_getreg(uint32_t imm) {
  return (imm & 63u) == 20u ? (uint32_t)(::simt::block_idx().x % 8u) : 0u;
}
#define __builtin_amdgcn_s_getreg(imm) simt_getreg((uint32_t)(imm))

// ---- runtime API (synchronous: every call completes before it returns,
// except for work recorded under stream capture, which a graph replays)
hipError_t hipGetDevice(int* d);
hipError_t hipSetDevice(int d);
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int d);
template <typename K>
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, K, int, size_t) {
  *n = 1;
  return hipSuccess;
}
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) {
  *p = const_cast<void*>(sym);
  return 0;
}
hipError_t hipGetLastError();
hipError_t hipPeekAtLastError();
const char* hipGetErrorString(hipError_t e);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind k, hipStream_t s);
hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind k);
hipError_t hipMemsetAsync(void* dst, int v, size_t n, hipStream_t s);
hipError_t hipHostMalloc(void** p, size_t n, unsigned flags);
hipError_t hipHostFree(void* p);
hipError_t hipMalloc(void** p, size_t n);
hipError_t hipFree(void* p);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamCreate(hipStream_t* s);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipDeviceSynchronize();
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode m);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t* err_node, char* log,
                               size_t log_len);
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t x);
hipError_t hipGraphDestroy(hipGraph_t g);
