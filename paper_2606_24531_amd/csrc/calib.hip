// Calibration kernels for the roofline measurements: they are not part of
// the decode path and the decode library does not link them.
//
// k_gather_lines reads whole 128-byte rows at given row indices, the access
// pattern of match sources in earlier blocks (short copies landing anywhere
// in the output), and either writes them out contiguously (copy) or folds
// them into one 16-byte value per thread (read only).  Eight lanes take one
// row, 16 bytes each, so one row is one 128-byte request.
#include <hip/hip_runtime.h>
#include <cstdint>

namespace {

constexpr uint32_t kThreads = 256;
constexpr uint32_t kUnroll = 4;  // rows in flight per lane

__global__ __launch_bounds__(kThreads) void k_gather_lines(const uint4* __restrict__ src, uint64_t src_rows,
                                                           const uint32_t* __restrict__ idx, uint64_t n,
                                                           uint4* __restrict__ dst, int read_only) {
  const uint64_t tid = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
  const uint32_t part = threadIdx.x & 7;
  const uint64_t stride = ((uint64_t)gridDim.x * kThreads) >> 3;  // rows per sweep of the grid
  uint4 acc = make_uint4(0, 0, 0, 0);
  for (uint64_t row = tid >> 3; row < n; row += kUnroll * stride) {
    uint4 v[kUnroll];
#pragma unroll
    for (uint32_t k = 0; k < kUnroll; k++) {
      const uint64_t r = row + k * stride;
      v[k] = make_uint4(0, 0, 0, 0);
      if (r < n) {
        const uint64_t j = idx[r];
        if (j < src_rows) v[k] = src[8 * j + part];
      }
    }
#pragma unroll
    for (uint32_t k = 0; k < kUnroll; k++) {
      const uint64_t r = row + k * stride;
      if (read_only) {
        acc.x ^= v[k].x;
        acc.y ^= v[k].y;
        acc.z ^= v[k].z;
        acc.w ^= v[k].w;
      } else if (r < n) {
        dst[8 * r + part] = v[k];
      }
    }
  }
  if (read_only) dst[tid] = acc;
}

}  // namespace

extern "C" {

// Threads one gather launch uses for `grid` workgroups (the read-only form
// writes one 16-byte value per thread, so dst must hold this many).
uint64_t acecalib_threads(uint32_t grid) { return (uint64_t)grid * kThreads; }

// Gathers n rows of 128 bytes: row i of the result is row idx[i] of src
// (src holds src_rows rows; an index at or past src_rows reads zeros).
// read_only = 0: dst (device, n * 128 bytes) receives the rows in order.
// read_only = 1: dst (device, acecalib_threads(grid) * 16 bytes) receives one
// XOR of the rows each thread read.  All pointers are device pointers,
// 16-byte aligned; the launch is asynchronous on `stream`.  Returns 0, or
// the HIP error code of the launch.
int acecalib_gather_lines(const void* src, uint64_t src_rows, const uint32_t* idx, uint64_t n, void* dst,
                          int read_only, uint32_t grid, hipStream_t stream) {
  if (!src || !idx || !dst || grid == 0) return (int)hipErrorInvalidValue;
  if (((uintptr_t)src | (uintptr_t)dst) & 15) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gather_lines, dim3(grid), dim3(kThreads), 0, stream, static_cast<const uint4*>(src),
                     src_rows, idx, n, static_cast<uint4*>(dst), read_only);
  return (int)hipGetLastError();
}

}  // extern "C"
