// Host entry points of the count and batch kernels of one genus G.  Each
// genus's kernels are built in a translation unit of their own
// (count_g1.hip .. count_g4.hip: an explicit instantiation of CountEntry<G>),
// so that the four compile in parallel; kernels.hip dispatches on g.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "plan.h"

namespace hwc {

template <int G>
struct CountEntry {
  // count_kernel<G, CT, WPE> over levels lo..hi (CT from coeff_bytes, the
  // register budget WPE = 1, 6 or 8 waves per SIMD from wpe); plog > 0 (with
  // a queue and every level): each tile's top level in 2^plog parts, their
  // counts summed in acc ([n][G], zeroed) and counted per tile in done
  static hipError_t launch(const PlanDesc& P, const PlanDesc* dP, int coeff_bytes, const void* codes,
                           const uint32_t* perm, const uint64_t* tiles, const uint32_t* ntiles, uint32_t* queue,
                           uint32_t lo, uint32_t hi, int32_t* outN, uint32_t* outLv, uint32_t plog, uint32_t* acc,
                           uint32_t* done, uint32_t grid, uint32_t block, uint32_t wpe, hipStream_t s);
  // batch_kernel<G> over njobs jobs, image slot of `slot` bytes
  static hipError_t batch(const JobDesc* jobs, uint32_t njobs, uint32_t slot, uint32_t grid, uint32_t block,
                          hipStream_t s);
  static hipError_t occupancy(int coeff_bytes, uint32_t block, uint32_t lds_bytes, uint32_t wpe, int* blocks_per_cu);
  static hipError_t occupancy_batch(uint32_t block, size_t lds_bytes, int* blocks_per_cu);
  // lets the kernels use the whole LDS image budget and checks that they
  // declare no static LDS (the table image must start at LDS address 0);
  // done once, outside any graph capture
  static hipError_t prepare();
};

}  // namespace hwc
