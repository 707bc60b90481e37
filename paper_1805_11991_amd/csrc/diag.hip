// Ceiling of the count kernel's bound, measured on the device it runs on.
//
// The count kernels spend their time in random 16-bit reads of the Zech
// logarithm tables (Sec. 3.2) held in LDS.  lds_gather_kernel performs only
// that access pattern: a table of E entries, each the byte offset of another
// pseudo-random entry, walked by CH independent dependent chains per lane on
// every lane of a full grid.  The rate it reaches is the practical ceiling
// the count kernel is compared against beside the HBM and MFMA peaks.
// dev_gather_kernel does the same over a u32 table in device memory, the
// placement of Zech tables too large for LDS.  valu_issue_kernel measures the
// other resource the count kernels saturate: the issue rate of plain 32-bit
// vector instructions.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.h"

namespace hwc {
namespace {

typedef __attribute__((address_space(3))) const uint16_t* gather_ptr;

__device__ __forceinline__ uint32_t mix32(uint32_t x) {   // xorshift-multiply integer hash
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

template <int CH>
__global__ __launch_bounds__(256) void lds_gather_kernel(uint32_t entries, uint32_t steps, uint32_t seed,
                                                         uint32_t odd, uint32_t* __restrict__ sink) {
  extern __shared__ uint32_t lds32[];
  uint16_t* tab = reinterpret_cast<uint16_t*>(lds32);
  for (uint32_t i = threadIdx.x; i < entries; i += blockDim.x)
    tab[i] = (uint16_t)(2u * (mix32(i ^ seed) % entries));
  __syncthreads();
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t a[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) a[c] = 2u * (mix32(gid * CH + c + seed) % entries);
  for (uint32_t s = 0; s < steps; ++s) {
#pragma unroll
    for (int c = 0; c < CH; ++c) a[c] = *(gather_ptr)(size_t)a[c];   // table at LDS address 0
  }
  uint32_t x = 0;
#pragma unroll
  for (int c = 0; c < CH; ++c) x ^= a[c];
  // every offset is even, so with an odd `odd` this store never happens; the
  // compiler cannot know that, and keeps every read
  if (x == odd) sink[0] = gid;
}

template <int CH>
hipError_t launch_ch(uint32_t entries, uint32_t steps, uint32_t grid, uint32_t bytes, uint32_t* sink,
                     hipStream_t s) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&lds_gather_kernel<CH>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsImageLimit);
  if (e != hipSuccess) return e;
  hipFuncAttributes fa;
  e = hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(&lds_gather_kernel<CH>));
  if (e != hipSuccess) return e;
  if (fa.sharedSizeBytes != 0) return hipErrorInvalidKernelFile;   // the table must start at address 0
  hipLaunchKernelGGL(lds_gather_kernel<CH>, dim3(grid), dim3(256), bytes, s, entries, steps, 12345u, 1u, sink);
  return hipGetLastError();
}

// The same walk over a u32 table in device memory (the placement of Zech
// tables too large for LDS, served by L2 and the MALL): entry i holds the
// index of another pseudo-random entry.
__global__ __launch_bounds__(256) void dev_table_fill_kernel(uint32_t* __restrict__ tab, uint32_t entries,
                                                             uint32_t seed) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < entries; i += gridDim.x * blockDim.x)
    tab[i] = mix32(i ^ seed) % entries;
}

template <int CH>
__global__ __launch_bounds__(256) void dev_gather_kernel(const uint32_t* __restrict__ tab, uint32_t entries,
                                                         uint32_t steps, uint32_t seed, uint32_t odd,
                                                         uint32_t* __restrict__ sink) {
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t a[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) a[c] = mix32(gid * CH + c + seed) % entries;
  for (uint32_t s = 0; s < steps; ++s) {
#pragma unroll
    for (int c = 0; c < CH; ++c) a[c] = tab[a[c]];
  }
  uint32_t x = 0;
#pragma unroll
  for (int c = 0; c < CH; ++c) x += a[c];
  // x < CH * entries <= 2^28 < odd (never true), which the compiler cannot see
  if (x == odd) sink[0] = gid;
}

template <int CH>
hipError_t launch_dev_ch(const uint32_t* tab, uint32_t entries, uint32_t steps, uint32_t grid, uint32_t* sink,
                         hipStream_t s) {
  hipLaunchKernelGGL(dev_gather_kernel<CH>, dim3(grid), dim3(256), 0, s, tab, entries, steps, 12345u, 0xFFFFFFFFu,
                     sink);
  return hipGetLastError();
}

// Eight independent chains per lane of a = min(a + b, a - c): three plain
// 32-bit VALU instructions per chain and step (v_add, v_sub, v_min), no
// dependence between the chains, 8 x 8 x 3 = 192 per loop iteration.
__global__ __launch_bounds__(256) void valu_issue_kernel(uint32_t iters, uint32_t b, uint32_t c, uint32_t odd,
                                                         uint32_t* __restrict__ sink) {
  uint32_t a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = (threadIdx.x * (k + 3)) ^ blockIdx.x;
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
#pragma unroll
      for (int k = 0; k < 8; ++k) a[k] = min(a[k] + b, a[k] - c);
    }
  }
  uint32_t x = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) x ^= a[k];
  if (x == odd && b == c) sink[0] = x;   // b != c in every launch: keeps the chains live
}

}  // namespace

hipError_t launch_valu_issue(uint32_t iters, uint32_t grid, uint32_t* sink, hipStream_t s) {
  if (grid == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(valu_issue_kernel, dim3(grid), dim3(256), 0, s, iters, 7u, 5u, 1u, sink);
  return hipGetLastError();
}

// tab: `entries` u32 of device memory, entries in [64, 2^26]
hipError_t launch_dev_table_fill(uint32_t* tab, uint32_t entries, hipStream_t s) {
  if (entries < 64 || entries > (1u << 26)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(dev_table_fill_kernel, dim3(1024), dim3(256), 0, s, tab, entries, 54321u);
  return hipGetLastError();
}

// chains 1, 2 or 4 over the table filled by launch_dev_table_fill; sink: one device u32
hipError_t launch_dev_gather(const uint32_t* tab, uint32_t entries, uint32_t chains, uint32_t steps, uint32_t grid,
                             uint32_t* sink, hipStream_t s) {
  if (entries < 64 || entries > (1u << 26) || grid == 0) return hipErrorInvalidValue;
  switch (chains) {
    case 1: return launch_dev_ch<1>(tab, entries, steps, grid, sink, s);
    case 2: return launch_dev_ch<2>(tab, entries, steps, grid, sink, s);
    case 4: return launch_dev_ch<4>(tab, entries, steps, grid, sink, s);
    default: return hipErrorInvalidValue;
  }
}

// entries in [64, kLdsImageLimit/2], chains 1, 2 or 4; sink: one device u32
hipError_t launch_lds_gather(uint32_t entries, uint32_t chains, uint32_t steps, uint32_t grid, uint32_t* sink,
                             hipStream_t s) {
  if (entries < 64 || entries > kLdsImageLimit / 2 || grid == 0) return hipErrorInvalidValue;
  const uint32_t bytes = (entries * 2u + 15u) & ~15u;
  switch (chains) {
    case 1: return launch_ch<1>(entries, steps, grid, bytes, sink, s);
    case 2: return launch_ch<2>(entries, steps, grid, bytes, sink, s);
    case 4: return launch_ch<4>(entries, steps, grid, bytes, sink, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hwc
