// Definitions of CountEntry<G> (count_entry.h), included only by the
// per-genus translation units count_g1.hip .. count_g4.hip.
#pragma once
#include "count_entry.h"
#include "count_impl.h"

namespace hwc {

template <int G>
hipError_t CountEntry<G>::launch(const PlanDesc& P, const PlanDesc* dP, int coeff_bytes, const void* codes,
                                 const uint32_t* perm, const uint64_t* tiles, const uint32_t* ntiles, uint32_t* queue,
                                 uint32_t lo, uint32_t hi, int32_t* outN, uint32_t* outLv, uint32_t plog,
                                 uint32_t* acc, uint32_t* done, uint32_t grid, uint32_t block, uint32_t wpe,
                                 hipStream_t s) {
#define HWC_LAUNCH(CT, W)                                                                                   \
  hipLaunchKernelGGL((count_kernel<G, CT, W>), dim3(grid), dim3(block), P.image_bytes, s, dP,                \
                     static_cast<const CT*>(codes), perm, tiles, ntiles, queue, lo, hi, outN, outLv, plog, acc, done)
  if (coeff_bytes == 1) {
    if (wpe >= 8) HWC_LAUNCH(int8_t, 8);
    else if (wpe >= 6) HWC_LAUNCH(int8_t, 6);
    else HWC_LAUNCH(int8_t, 1);
  } else {
    if (wpe >= 8) HWC_LAUNCH(int16_t, 8);
    else if (wpe >= 6) HWC_LAUNCH(int16_t, 6);
    else HWC_LAUNCH(int16_t, 1);
  }
#undef HWC_LAUNCH
  return hipGetLastError();
}

template <int G>
hipError_t CountEntry<G>::batch(const JobDesc* jobs, uint32_t njobs, uint32_t slot, uint32_t grid, uint32_t block,
                                hipStream_t s) {
  hipLaunchKernelGGL(batch_kernel<G>, dim3(grid), dim3(block), slot + 16, s, jobs, njobs, slot);
  return hipGetLastError();
}

template <int G>
hipError_t CountEntry<G>::occupancy(int coeff_bytes, uint32_t block, uint32_t lds_bytes, uint32_t wpe,
                                    int* blocks_per_cu) {
#define HWC_OCC(CT, W) \
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, count_kernel<G, CT, W>, block, lds_bytes)
  if (coeff_bytes == 1) {
    if (wpe >= 8) HWC_OCC(int8_t, 8);
    if (wpe >= 6) HWC_OCC(int8_t, 6);
    HWC_OCC(int8_t, 1);
  }
  if (wpe >= 8) HWC_OCC(int16_t, 8);
  if (wpe >= 6) HWC_OCC(int16_t, 6);
  HWC_OCC(int16_t, 1);
#undef HWC_OCC
}

template <int G>
hipError_t CountEntry<G>::occupancy_batch(uint32_t block, size_t lds_bytes, int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, batch_kernel<G>, block, lds_bytes);
}

template <int G>
hipError_t CountEntry<G>::prepare() {
  const void* counts[] = {reinterpret_cast<const void*>(&count_kernel<G, int8_t, 1>),
                          reinterpret_cast<const void*>(&count_kernel<G, int8_t, 6>),
                          reinterpret_cast<const void*>(&count_kernel<G, int8_t, 8>),
                          reinterpret_cast<const void*>(&count_kernel<G, int16_t, 1>),
                          reinterpret_cast<const void*>(&count_kernel<G, int16_t, 6>),
                          reinterpret_cast<const void*>(&count_kernel<G, int16_t, 8>)};
  const void* batch = reinterpret_cast<const void*>(&batch_kernel<G>);
  hipError_t e = hipSuccess;
  for (const void* f : counts)
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsImageLimit);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(batch, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsImageLimit + 16);
  auto no_static = [&](const void* f) {
    hipFuncAttributes a{};
    if (e == hipSuccess) e = hipFuncGetAttributes(&a, f);
    if (e == hipSuccess && a.sharedSizeBytes != 0) e = hipErrorInvalidKernelFile;
  };
  for (const void* f : counts) no_static(f);
  no_static(batch);
  return e;
}

}  // namespace hwc
