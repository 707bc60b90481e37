// Point counts by F_p-linear algebra on the matrix cores (prime q = p).
//
// For x in F_{p^j} = F_p[t]/(P) write x^i = sum_d a_{i,d} t^d.  Then f(x) =
// sum_i c_i x^i has coordinates D_d = sum_i c_i a_{i,d} (mod p): for a block of
// 32 swept points and 32 curves this is a 32 x 16 times 16 x 32 product of
// small integers, one v_mfma_i32_32x32x16_i8 per coordinate, exact in int32.
// The quadratic character of f(x) (Sec. 1.1: chi = 1, -1 or 0) then comes from
// one table read at the packed residues, so a (curve, point) pair costs the
// residues (a multiply, a shift and two multiply-adds per coordinate), one
// LDS read and one add -- against about 3.25 Zech reads and their
// bookkeeping per point in the logarithmic form.  The coefficients of one
// curve are the B operand (lane l holds curve l mod 32, coefficients
// 8 (l / 32) .. + 7), the points the A operand from LDS, and the result D has
// curve l mod 32 in every value of lane l (rows 8 (i/4) + 4 (l/32) + i mod 4),
// so each lane accumulates its own curve and two lanes are summed at the end.
// Rows need no bucketing: zero coefficients are just zeros in the product.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.h"

namespace hwc {
namespace {

typedef int v16i __attribute__((ext_vector_type(16)));
typedef const __attribute__((address_space(3))) uint16_t* vlds16_ptr;
typedef const __attribute__((address_space(3))) uint32_t* vlds32_ptr;
typedef const __attribute__((address_space(3))) uint64_t* vlds64_ptr;

__device__ __forceinline__ uint32_t vlds32(uint32_t a) { return *(vlds32_ptr)(size_t)a; }
__device__ __forceinline__ uint32_t vlds16(uint32_t a) { return *(vlds16_ptr)(size_t)a; }
__device__ __forceinline__ long vlds64(uint32_t a) { return (long)*(vlds64_ptr)(size_t)a; }

// c + a * b on 24-bit operands with b uniform, one instruction each (the
// compiler otherwise splits these into a multiply and a three-way add).  The
// hazard checks do not see into inline assembly, so no matrix-core result is
// read here first: every value is read by compiled code (its quotient) before,
// and the quotient is an input of these instructions, which orders them after.
__device__ __forceinline__ uint32_t mad_u24_after(uint32_t a, uint32_t b, uint32_t c, uint32_t after) {
  uint32_t r;
  asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c), "v"(after));
  return r;
}
__device__ __forceinline__ uint32_t mad_i24(uint32_t a, int32_t b, uint32_t c) {
  uint32_t r;
  asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
  return r;
}
__device__ __forceinline__ uint32_t quot(uint32_t v, uint32_t m, uint32_t s) {
  return (uint32_t)__umul24(v, m) >> s;
}
// floor(v m / 2^32) on 24-bit operands (v_mul_hi_u32_u24)
__device__ __forceinline__ uint32_t mulhi24(uint32_t v, uint32_t m) {
  return (uint32_t)(((uint64_t)(v & 0xFFFFFFu) * (m & 0xFFFFFFu)) >> 32);
}

// One level with KC coordinates: the lane's zeros and nonsquares over its rows.
// The character table has TW-byte entries; coordinate 0 comes scaled by TW
// from the matrix product, so its residue mod TW p is already TW r_0 (a byte
// offset).
template <int KC, int TW, bool BAL>
__device__ __forceinline__ void vlevel(const VLevel& L, uint32_t p, uint32_t sb, uint32_t lane, long b,
                                       uint32_t& zs, uint32_t& ns) {
  const uint32_t vrow = L.vo + (lane & 31u) * 16u + (lane >> 5) * 8u;
  // coordinate d >= 1 adds mult_d D_d - TW p^(d+1) q_d; in the balanced form
  // D_d carries a factor sb p, so its multiplier is TW p^(d-1) / sb
  const uint32_t mult1 = BAL ? TW / sb : TW * p, mult2 = BAL ? TW * p / sb : TW * p * p,
                 mult3 = BAL ? TW * p * p / sb : TW * p * p * p;
  const int32_t neg0 = -(int32_t)(TW * p), neg1 = -(int32_t)(TW * p * p), neg2 = -(int32_t)(TW * p * p * p),
                neg3 = -(int32_t)(TW * p * p * p * p);
  const v16i zero = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  uint32_t acc = 0;
#pragma unroll 1
  for (uint32_t bb = 0; bb < L.nblk; ++bb) {
    v16i D[KC];
#pragma unroll
    for (int d = 0; d < KC; ++d) {
      const long a = vlds64(vrow + (bb * KC + d) * 512u);
      D[d] = __builtin_amdgcn_mfma_i32_32x32x16_i8(a, b, zero, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      // v0 = table offset + 4 (coordinate 0); its quotient by 4p without the offset
      const uint32_t v0 = (uint32_t)D[0][i];
      const uint32_t q0 = ((uint32_t)__umul24(v0, L.m0) + L.nbm0) >> L.s0;
      uint32_t idx = mad_i24(q0, neg0, v0);
      if (KC > 1) {
        const uint32_t v = (uint32_t)D[1][i], q = BAL ? mulhi24(v, L.m1) : quot(v, L.m1, L.s1);
        idx = mad_i24(q, neg1, mad_u24_after(v, mult1, idx, q));
      }
      if (KC > 2) {
        const uint32_t v = (uint32_t)D[2][i], q = BAL ? mulhi24(v, L.m1) : quot(v, L.m1, L.s1);
        idx = mad_i24(q, neg2, mad_u24_after(v, mult2, idx, q));
      }
      if (KC > 3) {
        const uint32_t v = (uint32_t)D[3][i], q = BAL ? mulhi24(v, L.m1) : quot(v, L.m1, L.s1);
        idx = mad_i24(q, neg3, mad_u24_after(v, mult3, idx, q));
      }
      acc += TW == 4 ? vlds32(idx) : vlds16(idx);
    }
  }
  zs = acc >> 15;
  ns = acc & (kVZero - 1u);
}

// Level J (J + 1 coordinates) of a curve: lv[J] = zeros | nonsquares << 8,
// summed over the two lanes that hold the curve.
template <int J, int G, int TW, bool BAL>
__device__ __forceinline__ void level_counts(const VPlanDesc& V, uint32_t p, uint32_t sb, uint32_t lane, long b,
                                             uint32_t lvl_lo, uint32_t lvl_hi, uint32_t (&lv)[G]) {
  if constexpr (J < G) {
    if ((uint32_t)J < lvl_lo || (uint32_t)J > lvl_hi) return;
    const VLevel& L = V.lv[J];
    uint32_t zs, ns;
    vlevel<J + 1, TW, BAL>(L, p, sb, lane, b, zs, ns);
    zs += __shfl_xor(zs, 32);
    ns += __shfl_xor(ns, 32);
    zs -= L.pad;   // padding rows are zero points
    lv[J] = zs | (ns << 8);
  }
}

// ACC: the image holds part of the points (one pass of several); the counts
// are added to outLv (zeros | nonsquares << 8 per curve and level, which the
// assembly turns into N afterwards) and outN is not written.
template <int G, typename CT, int TW, bool ACC, bool BAL>
__global__ __launch_bounds__(1024) void vcount_kernel(const VPlanDesc* __restrict__ Vd, const CT* __restrict__ codes,
                                                      uint64_t n, uint32_t lvl_lo, uint32_t lvl_hi,
                                                      int32_t* __restrict__ outN, uint32_t* __restrict__ outLv,
                                                      uint32_t* __restrict__ err) {
  constexpr int NC = 2 * G + 3;
  const VPlanDesc& V = *Vd;
  extern __shared__ uint32_t vl32[];
  for (uint32_t i = threadIdx.x; i < V.image_bytes / 4; i += blockDim.x) vl32[i] = V.image[i];
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63u, half = lane >> 5;
  const uint32_t p = __builtin_amdgcn_readfirstlane(V.p), sb = __builtin_amdgcn_readfirstlane(V.sb);
  const uint64_t ntiles = (n + 31) / 32;
  const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  uint32_t bad = 0;
  for (uint64_t t = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; t < ntiles; t += nw) {
    const uint64_t row = t * 32 + (lane & 31u);
    const bool valid = row < n;
    uint32_t c[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      const int v = valid ? (int)codes[row * NC + i] : 0;
      if (v < 0 || v >= (int)p) bad |= 1u;
      c[i] = (v < 0 || v >= (int)p) ? 0u : (uint32_t)v;
    }
    if (valid && c[NC - 1] == 0 && c[NC - 2] == 0) bad |= 2u;
    // the B operand: codes, or sb times the balanced codes (as int8)
    uint32_t cb[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i)
      cb[i] = BAL ? (uint32_t)(sb * (int32_t)(2 * c[i] > p ? (int32_t)c[i] - (int32_t)p : (int32_t)c[i])) & 0xFFu
                  : c[i];
    long b = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t lo = j < NC ? cb[j < NC ? j : 0] : kVSlotUnit;
      const uint32_t hi = 8 + j < NC ? cb[8 + j < NC ? 8 + j : 0] : kVSlotUnit;
      b |= (long)(half ? hi : lo) << (8 * j);
    }
    uint32_t lv[G];
#pragma unroll
    for (int j = 0; j < G; ++j) lv[j] = 0;
    level_counts<0, G, TW, BAL>(V, p, sb, lane, b, lvl_lo, lvl_hi, lv);
    level_counts<1, G, TW, BAL>(V, p, sb, lane, b, lvl_lo, lvl_hi, lv);
    level_counts<2, G, TW, BAL>(V, p, sb, lane, b, lvl_lo, lvl_hi, lv);
    level_counts<3, G, TW, BAL>(V, p, sb, lane, b, lvl_lo, lvl_hi, lv);
    if (!valid || half) continue;
    if (ACC) {
#pragma unroll
      for (int j = 0; j < G; ++j)
        if ((uint32_t)j >= lvl_lo && (uint32_t)j <= lvl_hi) outLv[row * G + j] += lv[j];
      continue;
    }
    if (outLv) {
#pragma unroll
      for (int j = 0; j < G; ++j)
        if ((uint32_t)j >= lvl_lo && (uint32_t)j <= lvl_hi) outLv[row * G + j] = lv[j];
    }
    if (outN) {
      // x = 0 and the points at infinity (Sec. 1.1), then the levels
      const uint32_t to1 = V.lv[0].to;
      const uint32_t c0 = c[0], ct = c[NC - 1];
      const bool ns0 = vlds32(to1 + 4 * c0) == 1u, nst = vlds32(to1 + 4 * ct) == 1u;   // TW = 4 here
#pragma unroll
      for (int k = 1; k <= G; ++k) {
        const bool odd = k & 1;
        int32_t nk = (c0 == 0 ? 1 : (odd && ns0 ? 0 : 2)) + (ct == 0 ? 1 : (odd && nst ? 0 : 2));
        if (V.orbit) {
#pragma unroll
          for (int j = 1; j <= G; ++j) {
            if (k % j) continue;
            const uint32_t z = lv[j - 1] & 0xFFu, nsq = lv[j - 1] >> 8;
            const uint32_t sq = V.lv[j - 1].pts - z - nsq;
            const uint32_t s = ((k / j) % 2 == 0) ? sq + nsq : sq;
            nk += (int32_t)(j * z + 2 * j * s);
          }
        } else {
          const uint32_t z = lv[k - 1] & 0xFFu, nsq = lv[k - 1] >> 8;
          nk += (int32_t)(z + 2 * (V.lv[k - 1].pts - z - nsq));
        }
        outN[row * G + k - 1] = nk;
      }
    }
  }
  if (bad) atomicOr(err, bad);
}

}  // namespace

// tw: table entry bytes of the image (4, or 2 for a pass of a split level);
// acc: add the counts to outLv (a pass of several) instead of writing N.
hipError_t launch_vcount(const VPlanDesc& V, const VPlanDesc* dV, int coeff_bytes, const void* codes, uint64_t n,
                         uint32_t lvl_lo, uint32_t lvl_hi, uint32_t tw, bool acc, int32_t* outN, uint32_t* outLv,
                         uint32_t* err, uint32_t grid, uint32_t block, hipStream_t s) {
  const bool bal = V.bal != 0;
  if (n == 0) return hipSuccess;
  if (V.image_bytes > kLdsImageLimit || lvl_hi >= V.g || lvl_lo > lvl_hi) return hipErrorInvalidValue;
  if ((tw != 4 && tw != 2) || (tw == 2 && !acc) || (acc && !outLv)) return hipErrorInvalidValue;
#define HWC_VK(GG, CTT, TWV, ACCV)                                                                                \
  do {                                                                                                            \
    if (bal)                                                                                                      \
      hipLaunchKernelGGL((vcount_kernel<GG, CTT, TWV, ACCV, true>), dim3(grid), dim3(block), V.image_bytes, s, dV, \
                         static_cast<const CTT*>(codes), n, lvl_lo, lvl_hi, outN, outLv, err);                   \
    else                                                                                                          \
      hipLaunchKernelGGL((vcount_kernel<GG, CTT, TWV, ACCV, false>), dim3(grid), dim3(block), V.image_bytes, s,  \
                         dV, static_cast<const CTT*>(codes), n, lvl_lo, lvl_hi, outN, outLv, err);               \
  } while (0)
#define HWC_V(GG)                                                                                                 \
  case GG:                                                                                                        \
    if (coeff_bytes == 1) {                                                                                       \
      if (!acc) HWC_VK(GG, int8_t, 4, false);                                                                     \
      else if (tw == 4) HWC_VK(GG, int8_t, 4, true);                                                              \
      else HWC_VK(GG, int8_t, 2, true);                                                                           \
    } else {                                                                                                      \
      if (!acc) HWC_VK(GG, int16_t, 4, false);                                                                    \
      else if (tw == 4) HWC_VK(GG, int16_t, 4, true);                                                             \
      else HWC_VK(GG, int16_t, 2, true);                                                                          \
    }                                                                                                             \
    break;
  switch (V.g) {
    HWC_V(1) HWC_V(2) HWC_V(3) HWC_V(4)
    default: return hipErrorInvalidValue;
  }
#undef HWC_V
#undef HWC_VK
  return hipGetLastError();
}

// Largest dynamic LDS for every instantiation (none may declare static LDS:
// the image starts at address 0).
template <int G, typename CT, int TW, bool ACC>
hipError_t prepare_one() {
  hipError_t e = hipSuccess;
  for (const void* f : {reinterpret_cast<const void*>(&vcount_kernel<G, CT, TW, ACC, false>),
                        reinterpret_cast<const void*>(&vcount_kernel<G, CT, TW, ACC, true>)}) {
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsImageLimit);
    hipFuncAttributes fa;
    if (e == hipSuccess) e = hipFuncGetAttributes(&fa, f);
    if (e == hipSuccess && fa.sharedSizeBytes != 0) e = hipErrorInvalidKernelFile;
  }
  return e;
}

template <int G>
hipError_t prepare_g() {
  hipError_t e = prepare_one<G, int8_t, 4, false>();
  if (e == hipSuccess) e = prepare_one<G, int8_t, 4, true>();
  if (e == hipSuccess) e = prepare_one<G, int8_t, 2, true>();
  if (e == hipSuccess) e = prepare_one<G, int16_t, 4, false>();
  if (e == hipSuccess) e = prepare_one<G, int16_t, 4, true>();
  if (e == hipSuccess) e = prepare_one<G, int16_t, 2, true>();
  return e;
}

hipError_t prepare_vcount() {
  hipError_t e = prepare_g<1>();
  if (e == hipSuccess) e = prepare_g<2>();
  if (e == hipSuccess) e = prepare_g<3>();
  if (e == hipSuccess) e = prepare_g<4>();
  return e;
}

hipError_t occupancy_vcount(uint32_t g, uint32_t block, uint32_t lds_bytes, int* blocks_per_cu) {
  switch (g) {
    case 1: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, vcount_kernel<1, int8_t, 4, true, true>, block, lds_bytes);
    case 2: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, vcount_kernel<2, int8_t, 4, true, true>, block, lds_bytes);
    case 3: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, vcount_kernel<3, int8_t, 4, true, true>, block, lds_bytes);
    case 4: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, vcount_kernel<4, int8_t, 4, true, true>, block, lds_bytes);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hwc
