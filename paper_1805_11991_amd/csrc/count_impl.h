#pragma once
// Counting kernels for gfx950.
//
// Work layout.  One wave (64 lanes) counts 64 curves at once, one curve per
// lane, and all lanes walk the same list of x in F_{q^j} (x is uniform, so
// its log and every per-x quantity live in scalar registers).  Curves are
// first bucketed by degree and zero pattern so that a wave's Horner steps are
// uniform: zero coefficients become scalar branches, never lane divergence.
//
// Horner in relative log form.  For f = sum c_i X^i and x = gamma^L write
// P_i = c_i + x P_{i+1} (P_d = c_d) and A_i = log(P_i / c_i).  Then
//   A_i = Z(A_{i+1} + g_i L + log c_{i+1} - log c_i),
// with Z the Zech logarithm (eq. 2.1) and g_i the distance to the previous
// nonzero coefficient.  The per-curve constant log c_{i+1} - log c_i is
// precomputed per lane, so each step is one add of three registers and one
// table read from LDS.  A zero partial sum (1 + gamma^k = 0, the sentinel of
// table (3.2)) makes the next A equal log 1 = 0.  At the end
// f(x) = c_low x^low gamma^A, so f(x) = 0 iff A is the zero marker and the
// quadratic character is (-1)^(A + log c_low + low L) (M = |F^x| is even).
//
// Classification and reduction (eq. 3.3) happen in registers: each lane keeps
// per-level counts of zeros and of odd logs, split by the parity of low*L.
//
// This header holds the device code of the count (templates and inline
// functions only); each genus's kernels are instantiated in count_g<G>.hip.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "plan.h"

namespace hwc {

// LDS reads at absolute LDS byte addresses.  The count and batch kernels
// declare no static LDS, so their dynamic block -- the table image -- starts
// at address 0 (prepare_kernels checks this on the host), and a table step is
// one add and one read with no base to add.
typedef const __attribute__((address_space(3))) uint16_t* lds16_ptr;
typedef const __attribute__((address_space(3))) uint32_t* lds32_ptr;
__device__ __forceinline__ uint32_t lds_u16(uint32_t addr) { return *(lds16_ptr)(size_t)addr; }
__device__ __forceinline__ uint32_t lds_u32(uint32_t addr) { return *(lds32_ptr)(size_t)addr; }
constexpr uint32_t kImageBase = 0;   // LDS address of the dynamic block

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Uniform reads of data no kernel writes while it runs (x lists, tile words):
// through the constant address space they become scalar loads instead of
// vector loads that stall the wave on a full memory round trip.
typedef const __attribute__((address_space(4))) uint32_t* const_u32_ptr;
typedef const __attribute__((address_space(4))) uint64_t* const_u64_ptr;
__device__ __forceinline__ uint32_t sload(const uint32_t* p, uint32_t i) { return ((const_u32_ptr)p)[i]; }
__device__ __forceinline__ uint64_t sload64(const uint64_t* p, uint32_t i) { return ((const_u64_ptr)p)[i]; }
__device__ __forceinline__ LevelDesc load_level(const PlanDesc& P, uint32_t j) {
  static_assert(sizeof(LevelDesc) % 4 == 0, "LevelDesc is copied in dwords");
  LevelDesc L;
  const uint32_t* src = reinterpret_cast<const uint32_t*>(&P.lv[j]);
  uint32_t* dst = reinterpret_cast<uint32_t*>(&L);
#pragma unroll
  for (uint32_t i = 0; i < sizeof(LevelDesc) / 4; ++i) dst[i] = sload(src, i);
  return L;
}

// ----------------------------------------------------------------------------
// the count

struct LevelCounts {
  // zeros / odd logs over all swept points, and among the points whose
  // power low*L is odd (the others follow by difference); n1 = number of
  // those points.  Masks rather than selects keep the counters in registers.
  uint32_t zt, ot, z1, o1, n1;
  // n points of uniform class cls with z zeros and o odd logs
  __device__ __forceinline__ void add_n(uint32_t cls, uint32_t n, uint32_t z, uint32_t o) {
    const uint32_t m = 0u - (cls & 1u);
    zt += z;
    ot += o;
    z1 += z & m;
    o1 += o & m;
    n1 += n & m;
  }
  __device__ __forceinline__ void add(uint32_t cls, uint32_t z, uint32_t o) { add_n(cls, 1u, z, o); }
};

// Form A: byte-unit table, zero region; one add + one read per step.
// del[i] already holds 2*delta_i + table offset.  Returns the relative log
// (byte units, or the zero marker 6M) and the pending power low*x in pend.
template <int NC>
__device__ __forceinline__ uint32_t horner_a(const uint32_t (&del)[NC], uint32_t M, uint32_t d,
                                             uint32_t mask, uint32_t x, uint32_t& pend) {
  uint32_t a = 0, p = 0;
#pragma unroll
  for (int i = NC - 2; i >= 0; --i) {
    if ((uint32_t)i < d) {
      p += x; p = p >= M ? p - M : p;
      if ((mask >> i) & 1u) {
        a = lds_u16(a + del[i] + 2 * p);
        p = 0;
      }
    }
  }
  pend = p;
  return a;
}

// horner_a for two x at once: both chains advance inside one (uniform)
// branch per position, so their reads overlap.
template <int NC>
__device__ __forceinline__ void horner_a2(const uint32_t (&del)[NC], uint32_t M, uint32_t d, uint32_t mask,
                                          uint32_t x0, uint32_t x1, uint32_t& a0, uint32_t& a1, uint32_t& pend0,
                                          uint32_t& pend1) {
  uint32_t p0 = 0, p1 = 0;
  a0 = a1 = 0;
#pragma unroll
  for (int i = NC - 2; i >= 0; --i) {
    if ((uint32_t)i < d) {
      p0 += x0; p0 = p0 >= M ? p0 - M : p0;
      p1 += x1; p1 = p1 >= M ? p1 - M : p1;
      if ((mask >> i) & 1u) {
        a0 = lds_u16(a0 + del[i] + 2 * p0);
        a1 = lds_u16(a1 + del[i] + 2 * p1);
        p0 = p1 = 0;
      }
    }
  }
  pend0 = p0;
  pend1 = p1;
}

template <int NC, bool FULL, int D>
__device__ __forceinline__ void sweep_form_a(const uint32_t* xs, uint32_t nx, uint32_t M,
                                             const uint32_t (&del)[NC], uint32_t d, uint32_t mask, LevelCounts& c) {
  const uint32_t S = 6 * M;
  uint32_t ix = 0;
  uint32_t n0 = 0, n1 = 1;
  if (xs && nx >= 2) { n0 = sload(xs, 0); n1 = sload(xs, 1); }
  for (; ix + 2 <= nx; ix += 2) {
    const uint32_t x0 = n0, x1 = n1;
    if (ix + 4 <= nx) {   // next pair, loaded while this one runs
      n0 = xs ? sload(xs, ix + 2) : ix + 2;
      n1 = xs ? sload(xs, ix + 3) : ix + 3;
    } else if (ix + 3 <= nx) {
      n0 = xs ? sload(xs, ix + 2) : ix + 2;
    }
    if (FULL) {
      uint32_t a0 = 0, a1 = 0;
      const uint32_t b0 = 2 * x0, b1 = 2 * x1;
#pragma unroll
      for (int i = D - 1; i >= 0; --i) {
        a0 = lds_u16(a0 + del[i] + b0);
        a1 = lds_u16(a1 + del[i] + b1);
      }
      c.zt += (a0 == S) + (a1 == S);
      c.ot += ((a0 >> 1) & 1u) + ((a1 >> 1) & 1u);
    } else {
      uint32_t p0, p1, a0, a1;
      horner_a2<NC>(del, M, d, mask, x0, x1, a0, a1, p0, p1);
      c.add(p0 & 1u, a0 == S, (a0 >> 1) & 1u);
      c.add(p1 & 1u, a1 == S, (a1 >> 1) & 1u);
    }
  }
  if (ix < nx) {
    const uint32_t x0 = xs ? sload(xs, ix) : ix;
    uint32_t p0;
    const uint32_t a0 = horner_a<NC>(del, M, d, mask, x0, p0);
    c.add(p0 & 1u, a0 == S, (a0 >> 1) & 1u);
  }
}

__device__ __forceinline__ uint32_t addmod(uint32_t a, uint32_t b, uint32_t M) {  // a, b < M
  const uint32_t s = a + b;
  return s >= M ? s - M : s;
}

// Sub-polynomial r of the split (positions i = r mod MS) by relative Horner in
// y (log Y).  sup has bit d set.  Returns the relative log (byte units or the
// zero marker) and in pend the power t_r Y of the class's lowest term.
template <int NC, int MS, int R, bool FULL, int D>
__device__ __forceinline__ uint32_t horner_class(const uint32_t (&sdel)[NC], uint32_t M,
                                                 uint32_t d, uint32_t sup, uint32_t Y, uint32_t& pend) {
  uint32_t a = 0;
  if (FULL) {  // every position 0..D holds a term: steps of one power of y
    const uint32_t b = 2 * Y;
    constexpr int TOP = D - ((D - R) % MS);
#pragma unroll
    for (int i = TOP - MS; i >= 0; i -= MS) a = lds_u16(a + sdel[i] + b);
    pend = 0;
    return a;
  }
  uint32_t p = 0;
  bool started = false;
#pragma unroll
  for (int i = NC - 1; i >= 0; --i) {
    if (i % MS != R) continue;
    if ((uint32_t)i > d) continue;
    if (started) p = addmod(p, Y, M);
    if ((sup >> i) & 1u) {
      if (started) a = lds_u16(a + sdel[i] + 2 * p);
      started = true;
      p = 0;
    }
  }
  pend = p;
  return a;
}

// The MS sub-polynomials of a sparse row (form A) in one pass over the
// positions from the top: every position issues its read, so the classes'
// reads overlap in straight-line code.  A position without a term, or the top
// term of its class, reads the table's first entry on every lane (sdel of the
// top position is the bare table offset) and discards it: one address for
// the whole wave, so the LDS serves it as a broadcast, with no bank conflicts.
template <int NC, int MS>
__device__ __forceinline__ void horner_classes_a(const uint32_t (&sdel)[NC], uint32_t M, uint32_t d, uint32_t sup,
                                                 uint32_t Y, uint32_t (&a)[4], uint32_t (&pend)[4]) {
  uint32_t p[4] = {0, 0, 0, 0};
  bool st[4] = {false, false, false, false};
#pragma unroll
  for (int r = 0; r < 4; ++r) a[r] = 0;
#pragma unroll
  for (int i = NC - 1; i >= 0; --i) {
    const int r = i % MS;
    if ((uint32_t)i > d) continue;
    const bool present = (sup >> i) & 1u;
    if (st[r]) p[r] = addmod(p[r], Y, M);
    const bool go = present && st[r];
    const uint32_t v = lds_u16(go ? a[r] + sdel[i] + 2 * p[r] : sdel[NC - 1]);
    a[r] = go ? v : a[r];
    if (present) {
      st[r] = true;
      p[r] = 0;
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) pend[r] = p[r];
}

// Per-curve constants of the split on one level: ll[r] = log of the lowest
// coefficient of class r, blane = parity of the lowest coefficient's log.
struct SplitConst {
  uint32_t ll[4];
  uint32_t blane;
};

__device__ __forceinline__ uint32_t submod(uint32_t a, uint32_t b, uint32_t M) {  // a, b < M
  return a >= b ? a - b : a + M - b;
}

// Zero-safe sum of two field elements given as absolute logs in byte units
// (2 log, in [0, 2M)) or the zero marker S: one read of the table's first
// 2M bytes (2 Z(k), or S where 1 + gamma^k = 0).
__device__ __forceinline__ uint32_t zadd(uint32_t tab, uint32_t M2, uint32_t S, uint32_t u,
                                         uint32_t v) {
  const bool uz = u == S, vz = v == S;
  uint32_t d = v - u;
  d = min(d, d + M2);
  const uint32_t r = lds_u16(tab + ((uz || vz) ? 0u : d));
  uint32_t s = u + r;
  s = min(s, s - M2);
  return uz ? v : (vz ? u : (r == S ? S : s));
}

__device__ __forceinline__ uint32_t zmul(uint32_t v, uint32_t k, uint32_t M2, uint32_t S) {  // k < 2M bytes
  uint32_t s = v + k;
  s = min(s, s - M2);
  return v == S ? S : s;
}

// Split evaluation over mu_MS cosets (form A).  With w = gamma^(M/MS) in F_q,
// f(w^s x) = sum_r w^(s r) x^r f_r(x^MS): the MS points of a tuple share the
// sub-polynomial values at y = x^MS.
//   MS = 2, 3: the MS - 1 Zech additions per point chain from the top class
//     in relative form, B = Z(a_2 - a_1), R = Z(B + a_1 - a_0), log f = R + a_0
//     (a_r = log(w^(s r) x^r f_r(y))).  A vanishing f_r(y) below the top
//     class has no relative log; the wave then evaluates the tuple's points
//     by plain Horner.
//   MS = 4 (4 | q - 1): two radix-2 stages, f(x) = E(x^2) + x O(x^2) with
//     E(v) = f_0(v^2) + v f_2(v^2), O(v) = f_1(v^2) + v f_3(v^2); the points
//     x, -x share E(x^2), O(x^2), and ix, -ix share E(-x^2), O(-x^2): four
//     additions for E and O, one per point.  Relative form as above; when a
//     base vanishes (f_0(y), f_1(y) or E) the wave redoes the eight additions
//     zero-safe on absolute logs.
template <int NC, int MS, bool FULL, int D>
__device__ __forceinline__ void sweep_split_a(const LevelDesc& L, const uint32_t (&sdel)[NC],
                                              const uint32_t (&del)[NC], uint32_t d, uint32_t mask,
                                              const SplitConst& K, LevelCounts& c) {
  const uint32_t M = L.M, M2 = 2 * M, S = 6 * M, step = M / MS, tab = L.tab_off;
  const uint32_t dl1 = submod(K.ll[1], K.ll[0], M);
  const uint32_t K1 = M2 + 2 * dl1;
  const uint32_t K2 = M2 + 2 * (MS == 4 ? submod(K.ll[2], K.ll[0], M) : submod(K.ll[2], K.ll[1], M));
  const uint32_t K3 = M2 + 2 * submod(K.ll[3], K.ll[1], M);
  const uint32_t fix = (K.ll[0] ^ K.blane) & 1u;
  const uint32_t sup = mask | (1u << d);
  const uint32_t nt = L.nt;
  const uint32_t* xt = L.xs_t;
  uint32_t xnext = (xt && nt) ? sload(xt, 0) : 0u;
  for (uint32_t it = 0; it < nt; ++it) {
    const uint32_t x = xnext;
    if (it + 1 < nt) xnext = xt ? sload(xt, it + 1) : it + 1;
    uint32_t Y = 0;
#pragma unroll
    for (int m = 0; m < MS; ++m) Y = addmod(Y, x, M);
    uint32_t p0, p1, p2 = 0, p3 = 0;
    uint32_t a0, a1, a2 = S, a3 = S;
    if (FULL) {
      a0 = horner_class<NC, MS, 0, FULL, D>(sdel, M, d, sup, Y, p0);
      a1 = horner_class<NC, MS, 1, FULL, D>(sdel, M, d, sup, Y, p1);
      if (MS >= 3) a2 = horner_class<NC, MS, 2, FULL, D>(sdel, M, d, sup, Y, p2);
      if (MS == 4) a3 = horner_class<NC, MS, 3, FULL, D>(sdel, M, d, sup, Y, p3);
    } else {
      uint32_t av[4], pv[4];
      horner_classes_a<NC, MS>(sdel, M, d, sup, Y, av, pv);
      a0 = av[0]; a1 = av[1]; p0 = pv[0]; p1 = pv[1];
      if (MS >= 3) { a2 = av[2]; p2 = pv[2]; }
      if (MS == 4) { a3 = av[3]; p3 = pv[3]; }
    }
    const uint32_t cls = FULL ? 0u : (p0 & 1u);  // parity of t_0 Y
    if (MS == 4) {
      const uint32_t x2 = addmod(x, x, M), h = M / 2;
      const uint32_t uE = addmod(addmod(x2, p2, M), p0 ? M - p0 : 0u, M);
      const uint32_t uO = addmod(addmod(x2, p3, M), p1 ? M - p1 : 0u, M);
      const uint32_t vf = addmod(addmod(x, p1, M), p0 ? M - p0 : 0u, M);
      // clamped bases keep every index in the table while the wave decides
      const bool base_zero = (a0 == S) || (a1 == S);
      const uint32_t b0 = base_zero ? 0u : a0, b1 = base_zero ? 0u : a1;
      uint32_t FE = K2 - b0;                          // (0, 4M)
      FE = min(FE, FE - M2);
      uint32_t FO = K3 - b1;
      FO = min(FO, FO - M2);
      const uint32_t Ep = lds_u16(a2 + FE + 2 * uE + tab);
      const uint32_t Em = lds_u16(a2 + FE + 2 * addmod(uE, h, M) + tab);
      const uint32_t Op = lds_u16(a3 + FO + 2 * uO + tab);
      const uint32_t Om = lds_u16(a3 + FO + 2 * addmod(uO, h, M) + tab);
      uint32_t u = 0, zs = 0, odd;
      if (!__ballot(base_zero || Ep == S || Em == S)) {
        uint32_t G = b1 + K1 - b0;                    // (0, 6M)
        G = min(G, G - M2);
        G = min(G, G - M2);
        G += M2;
        // bit 1 of E + r (both even) is bit 1 of E ^ r; a zero point (r = S)
        // must not count, which the rare branch below takes care of
        uint32_t r[4];
        bool anyz = false;
#pragma unroll
        for (uint32_t s = 0; s < 4; ++s) {
          const uint32_t E = (s & 1u) ? Em : Ep;
          const uint32_t O = (s & 1u) ? Om : Op;
          uint32_t F = G - E;                         // (0, 4M)
          F = min(F, F - M2);
          r[s] = lds_u16(O + F + 2 * addmod(vf, s * step, M) + tab);
          u += (E ^ r[s]) & 2u;
          anyz |= r[s] == S;
        }
        if (__ballot(anyz)) {
          u = 0;
#pragma unroll
          for (uint32_t s = 0; s < 4; ++s) {
            const uint32_t E = (s & 1u) ? Em : Ep;
            const bool z = r[s] == S;
            zs += z;
            u += z ? 0u : ((E ^ r[s]) & 2u);
          }
        }
        u >>= 1;
        odd = ((a0 >> 1) ^ fix) & 1u ? (4 - zs) - u : u;
      } else {
        // absolute logs (byte units) of f_r(y) w^.. x^..: 2 (ll_r + p_r) + a_r
        const uint32_t v0 = zmul(a0, 2 * addmod(K.ll[0], p0, M), M2, S);
        const uint32_t v1 = zmul(a1, 2 * addmod(K.ll[1], p1, M), M2, S);
        const uint32_t v2 = zmul(a2, 2 * addmod(K.ll[2], p2, M), M2, S);
        const uint32_t v3 = zmul(a3, 2 * addmod(K.ll[3], p3, M), M2, S);
        const uint32_t ep = zadd(tab, M2, S, v0, zmul(v2, 2 * x2, M2, S));
        const uint32_t em = zadd(tab, M2, S, v0, zmul(v2, 2 * addmod(x2, h, M), M2, S));
        const uint32_t op = zadd(tab, M2, S, v1, zmul(v3, 2 * x2, M2, S));
        const uint32_t om = zadd(tab, M2, S, v1, zmul(v3, 2 * addmod(x2, h, M), M2, S));
        odd = 0;
#pragma unroll
        for (uint32_t s = 0; s < 4; ++s) {
          const uint32_t E = (s & 1u) ? em : ep;
          const uint32_t O = (s & 1u) ? om : op;
          const uint32_t f = zadd(tab, M2, S, E, zmul(O, 2 * addmod(x, s * step, M), M2, S));
          const bool z = f == S;
          zs += z;
          // A = log f - log c_low - t_0 Y
          odd += z ? 0u : (((f >> 1) ^ K.blane ^ cls) & 1u);
        }
      }
      c.add_n(cls, 4, zs, odd);
      continue;
    }
    const bool inner_zero = (a0 == S) || (MS == 3 && a1 == S);
    if (__ballot(inner_zero)) {
      for (uint32_t s = 0; s < MS; ++s) {
        uint32_t pp;
        const uint32_t xs = addmod(x, s * step, M);
        const uint32_t a = horner_a<NC>(del, M, d, mask, xs, pp);
        c.add(pp & 1u, a == S, (a >> 1) & 1u);
      }
      continue;
    }
    // zero values contribute bit 1 of 6M = 0; the lane's parity (a0 + fix) is
    // applied once per tuple: odd = u if even, else (non-zero points) - u
    uint32_t u = 0, zs = 0;
    if (MS == 2) {
      uint32_t F1 = K1 - a0;                          // (0, 4M)
      F1 = min(F1, F1 - 2 * M);
      const uint32_t v1 = addmod(addmod(x, p1, M), p0 ? M - p0 : 0u, M);
#pragma unroll
      for (uint32_t s = 0; s < 2; ++s) {
        const uint32_t w1 = 2 * addmod(v1, s * step, M) + tab;
        const uint32_t r = lds_u16(a1 + F1 + w1);
        u += r & 2u;
        zs += r == S;
      }
    } else {
      uint32_t F2 = K2 - a1;                          // (0, 4M)
      F2 = min(F2, F2 - 2 * M);
      uint32_t F1 = a1 + K1 - a0;                     // (0, 6M)
      F1 = min(F1, F1 - 2 * M);
      F1 = min(F1, F1 - 2 * M);
      const uint32_t v2 = addmod(addmod(x, p2, M), p1 ? M - p1 : 0u, M);
      const uint32_t v1 = addmod(addmod(x, p1, M), p0 ? M - p0 : 0u, M);
#pragma unroll
      for (uint32_t s = 0; s < 3; ++s) {
        const uint32_t w2 = 2 * addmod(v2, s * step, M) + tab;
        const uint32_t w1 = 2 * addmod(v1, s * step, M) + tab;
        const uint32_t b = lds_u16(a2 + F2 + w2);
        const uint32_t r = lds_u16(b + F1 + w1);
        u += r & 2u;
        zs += r == S;
      }
    }
    u >>= 1;
    const uint32_t odd = ((a0 >> 1) ^ fix) & 1u ? (MS - zs) - u : u;
    c.add_n(cls, MS, zs, odd);
  }
}

__device__ __forceinline__ uint32_t fold(uint32_t v, uint32_t M) { return min(v, v - M); }  // [0, 2M) -> [0, M)

// Table modes of the element-unit levels: kTabC (form C: two periods of 2 Z in
// LDS), kTabD (form D: the same as u32 in device memory), kTabE (form E: one
// period of Z in LDS, u16 entries for M <= 65534), kTabF (form F: half a
// period of 17-bit Z in LDS, M <= 131070), kTabG (form G: the same half period
// as u32 entries in byte units, where it fits).
constexpr int kTabC = 0, kTabD = 1, kTabE = 2, kTabF = 3, kTabG = 4;

// Table entry at byte offset r in [0, 2 M2) (M2 = 2 M, the byte period):
// 2 Z((r/2) mod M), or the marker M2 where 1 + gamma^(r/2) = 0.  Form E folds
// the offset into its one period and doubles the entry it reads (its marker M
// becomes M2).
template <int TM>
__device__ __forceinline__ uint32_t tab_c(uint32_t tab, const uint32_t* __restrict__ gtab, uint32_t M2, uint32_t r) {
  if (TM == kTabD) return gtab[r >> 1];
  if (TM == kTabE) return 2u * lds_u16(tab + fold(r, M2));
  if (TM == kTabF) {
    // element k of one period; past the half, Z(k) = Z(M - k) + k mod M
    const uint32_t M = M2 >> 1, h = M2 >> 2;
    const uint32_t k = fold(r, M2) >> 1;
    const bool up = k > h;
    const uint32_t j = up ? M - k : k;                                    // j <= h
    const uint32_t bits = tab + ((2u * (h + 1u) + 15u) & ~15u);           // the 17th bits after the low halves
    const uint32_t z = lds_u16(tab + 2u * j) | (((lds_u32(bits + 4u * (j >> 5)) >> (j & 31u)) & 1u) << 16);
    // Z(k) is never 0 (1 + gamma^k = 1 has no solution), so the sum is
    // reduced into [1, M] instead of [0, M): the same value for every entry,
    // and the marker M (at j = h, not mirrored) stays M, i.e. M2 in bytes
    const uint32_t y = z + (up ? k : 0u) - 1u;                            // < 2M - 1
    return 2u * fold(y, M) + 2u;
  }
  if (TM == kTabG) {
    // entries 2 Z(j), j <= M/2, and 2 M2 at j = M/2 (the marker, which the
    // final fold turns into M2); past the half, 2 Z(k) = 2 Z(M - k) + 2k mod M2
    const uint32_t rr = fold(r, M2);                                      // 2k
    const bool up = rr > (M2 >> 1);
    const uint32_t z2 = lds_u32(tab + 2u * (up ? M2 - rr : rr));
    return fold(z2 + (up ? rr : 0u), M2);
  }
  return lds_u16(tab + r);
}

// Forms C, D and E work in byte units like form A: every log, delta and power
// is doubled, the period is M2 = 2M and the zero marker is M2, so a folded
// index is the byte offset of the entry (form C's table sits at the start of
// the LDS image) and a log's parity is its bit 1.  In the functions below
// the parameter M is this byte period.
//
// Form C/D relative Horner for two x at once (index folded into the table's
// two periods; reads of both chains inside one uniform branch per position).
// Not EXACT: a vanishing partial sum sets hit and the caller redoes the pair
// with EXACT, which restarts from the coefficient.
template <int NC, bool EXACT, int TM>
__device__ __forceinline__ void horner_c2(uint32_t tab, const uint32_t* __restrict__ gtab, uint32_t M,
                                          const uint32_t (&del)[NC], uint32_t d, uint32_t mask, uint32_t x0,
                                          uint32_t x1, uint32_t& a0, uint32_t& a1, uint32_t& pend0, uint32_t& pend1,
                                          bool& hit) {
  uint32_t p0 = 0, p1 = 0;
  a0 = a1 = 0;
#pragma unroll
  for (int i = NC - 2; i >= 0; --i) {
    if ((uint32_t)i < d) {
      p0 += x0; p0 = p0 >= M ? p0 - M : p0;
      p1 += x1; p1 = p1 >= M ? p1 - M : p1;
      if ((mask >> i) & 1u) {
        const uint32_t r0 = min(a0 + del[i] + p0, a0 + del[i] + p0 - M);   // < 2M
        const uint32_t r1 = min(a1 + del[i] + p1, a1 + del[i] + p1 - M);
        const uint32_t v0 = tab_c<TM>(tab, gtab, M, r0);
        const uint32_t v1 = tab_c<TM>(tab, gtab, M, r1);
        if (EXACT) {
          a0 = (a0 == M) ? 0u : v0;
          a1 = (a1 == M) ? 0u : v1;
        } else {
          hit |= (v0 == M) | (v1 == M);
          a0 = v0;
          a1 = v1;
        }
        p0 = p1 = 0;
      }
    }
  }
  pend0 = p0;
  pend1 = p1;
}

template <int NC, int TM>
__device__ __forceinline__ void sweep_form_c(const LevelDesc& L, const uint32_t* xs, uint32_t nx,
                                             const uint32_t (&del)[NC], uint32_t d, uint32_t mask, LevelCounts& c) {
  const uint32_t M = 2 * L.M, tab = L.tab_off;
  const uint32_t* gtab = L.gtab;
  uint32_t delb[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) delb[i] = 2 * del[i];
  for (uint32_t ix = 0; ix < nx; ix += 2) {
    const uint32_t x0 = 2 * (xs ? sload(xs, ix) : ix);
    const bool two = ix + 1 < nx;
    const uint32_t x1 = two ? 2 * (xs ? sload(xs, ix + 1) : ix + 1) : x0;
    bool hit = false;
    uint32_t p0, p1, a0, a1;
    horner_c2<NC, false, TM>(tab, gtab, M, delb, d, mask, x0, x1, a0, a1, p0, p1, hit);
    if (__ballot(hit)) horner_c2<NC, true, TM>(tab, gtab, M, delb, d, mask, x0, x1, a0, a1, p0, p1, hit);
    c.add((p0 >> 1) & 1u, a0 == M, (a0 >> 1) & 1u);   // bit 1 of the marker 2M is 0
    if (two) c.add((p1 >> 1) & 1u, a1 == M, (a1 >> 1) & 1u);
  }
}


// Sub-polynomial r of the split on a form C/D level (byte units): as
// horner_class, with the index folded into the table's two periods.  Not
// EXACT: a vanishing partial sum sets hit (the caller redoes the tuple).
template <int NC, int MS, int R, bool FULL, int D, bool EXACT, int TM>
__device__ __forceinline__ uint32_t horner_class_c(uint32_t tab, const uint32_t* __restrict__ gtab,
                                                   const uint32_t (&sdel)[NC], uint32_t M, uint32_t d, uint32_t sup,
                                                   uint32_t Y, uint32_t& pend, bool& hit) {
  uint32_t a = 0;
  if (FULL) {
    constexpr int TOP = D - ((D - R) % MS);
#pragma unroll
    for (int i = TOP - MS; i >= 0; i -= MS) {
      // index < 3M, folded below 2M, which every form reads; the first step
      // (a = 0) is below 2M already
      const uint32_t r = (i == TOP - MS) ? sdel[i] + Y : fold(a + sdel[i] + Y, M);
      const uint32_t v = tab_c<TM>(tab, gtab, M, r);
      if (EXACT) a = (a == M) ? 0u : v;
      else { hit |= v == M; a = v; }
    }
    pend = 0;
    return a;
  }
  uint32_t p = 0;
  bool started = false;
#pragma unroll
  for (int i = NC - 1; i >= 0; --i) {
    if (i % MS != R) continue;
    if ((uint32_t)i > d) continue;
    if (started) p = addmod(p, Y, M);
    if ((sup >> i) & 1u) {
      if (started) {
        const uint32_t v = tab_c<TM>(tab, gtab, M, fold(a + sdel[i] + p, M));
        if (EXACT) a = (a == M) ? 0u : v;
        else { hit |= v == M; a = v; }
      }
      started = true;
      p = 0;
    }
  }
  pend = p;
  return a;
}

// The MS sub-polynomials of a sparse row on a form C/D level in one pass
// (as horner_classes_a); not EXACT: a vanishing partial sum sets hit.
template <int NC, int MS, bool EXACT, int TM>
__device__ __forceinline__ void horner_classes_c(uint32_t tab, const uint32_t* __restrict__ gtab,
                                                 const uint32_t (&sdel)[NC], uint32_t M, uint32_t d, uint32_t sup,
                                                 uint32_t Y, uint32_t (&a)[4], uint32_t (&pend)[4], bool& hit) {
  uint32_t p[4] = {0, 0, 0, 0};
  bool st[4] = {false, false, false, false};
#pragma unroll
  for (int r = 0; r < 4; ++r) a[r] = 0;
#pragma unroll
  for (int i = NC - 1; i >= 0; --i) {
    const int r = i % MS;
    if ((uint32_t)i > d) continue;
    const bool present = (sup >> i) & 1u;
    if (st[r]) p[r] = addmod(p[r], Y, M);
    const bool go = present && st[r];
    // a position that does not step reads entry 0 on every lane (a broadcast)
    const uint32_t v = tab_c<TM>(tab, gtab, M, go ? fold(a[r] + sdel[i] + p[r], M) : 0u);
    if (EXACT) a[r] = go ? ((a[r] == M) ? 0u : v) : a[r];
    else {
      hit |= go && v == M;
      a[r] = go ? v : a[r];
    }
    if (present) {
      st[r] = true;
      p[r] = 0;
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) pend[r] = p[r];
}

// Zero-safe sum (absolute logs in [0, M) or the zero marker M, byte units).
template <int TM>
__device__ __forceinline__ uint32_t zadd_c(uint32_t tab, const uint32_t* __restrict__ gtab, uint32_t M, uint32_t u,
                                           uint32_t v) {
  const bool uz = u == M, vz = v == M;
  uint32_t dd = v - u;
  dd = min(dd, dd + M);
  const uint32_t r = tab_c<TM>(tab, gtab, M, (uz || vz) ? 0u : dd);
  const uint32_t s = fold(u + r, M);
  return uz ? v : (vz ? u : (r == M ? M : s));
}

__device__ __forceinline__ uint32_t zmul_c(uint32_t v, uint32_t k, uint32_t M) {  // k < M
  return v == M ? M : fold(v + k, M);
}

// Radix-2x2 split over mu_4 cosets on a form C/D level: the same stages as the
// MS = 4 case of sweep_split_a (byte units, K.ll doubled by the caller).
template <int NC, bool FULL, int D, int TM>
__device__ __forceinline__ void sweep_split_c(const LevelDesc& L, const uint32_t (&sdel_e)[NC], uint32_t d,
                                              uint32_t mask, const SplitConst& Ke, LevelCounts& c) {
  uint32_t sdel[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) sdel[i] = 2 * sdel_e[i];
  SplitConst K = Ke;
#pragma unroll
  for (int r = 0; r < 4; ++r) K.ll[r] = 2 * Ke.ll[r];
  const uint32_t M = 2 * L.M, step = M / 4, tab = L.tab_off, h = M / 2;
  const uint32_t* gtab = L.gtab;
  const uint32_t K1 = M + submod(K.ll[1], K.ll[0], M);
  const uint32_t K2 = M + submod(K.ll[2], K.ll[0], M);
  const uint32_t K3 = M + submod(K.ll[3], K.ll[1], M);
  const uint32_t fix = ((K.ll[0] >> 1) ^ K.blane) & 1u;
  const uint32_t sup = mask | (1u << d);
  const uint32_t nt = L.nt;
  const uint32_t* xt = L.xs_t;
  uint32_t xnext = (xt && nt) ? sload(xt, 0) : 0u;
  for (uint32_t it = 0; it < nt; ++it) {
    const uint32_t x = 2 * xnext;
    if (it + 1 < nt) xnext = xt ? sload(xt, it + 1) : it + 1;
    const uint32_t x2 = addmod(x, x, M);
    const uint32_t Y = addmod(x2, x2, M);
    uint32_t p0, p1, p2, p3;
    uint32_t a0, a1, a2, a3;
    bool hit = false;
    if (FULL) {
      a0 = horner_class_c<NC, 4, 0, FULL, D, false, TM>(tab, gtab, sdel, M, d, sup, Y, p0, hit);
      a1 = horner_class_c<NC, 4, 1, FULL, D, false, TM>(tab, gtab, sdel, M, d, sup, Y, p1, hit);
      a2 = horner_class_c<NC, 4, 2, FULL, D, false, TM>(tab, gtab, sdel, M, d, sup, Y, p2, hit);
      a3 = horner_class_c<NC, 4, 3, FULL, D, false, TM>(tab, gtab, sdel, M, d, sup, Y, p3, hit);
      if (__ballot(hit)) {
        a0 = horner_class_c<NC, 4, 0, FULL, D, true, TM>(tab, gtab, sdel, M, d, sup, Y, p0, hit);
        a1 = horner_class_c<NC, 4, 1, FULL, D, true, TM>(tab, gtab, sdel, M, d, sup, Y, p1, hit);
        a2 = horner_class_c<NC, 4, 2, FULL, D, true, TM>(tab, gtab, sdel, M, d, sup, Y, p2, hit);
        a3 = horner_class_c<NC, 4, 3, FULL, D, true, TM>(tab, gtab, sdel, M, d, sup, Y, p3, hit);
      }
    } else {
      uint32_t av[4], pv[4];
      horner_classes_c<NC, 4, false, TM>(tab, gtab, sdel, M, d, sup, Y, av, pv, hit);
      if (__ballot(hit)) horner_classes_c<NC, 4, true, TM>(tab, gtab, sdel, M, d, sup, Y, av, pv, hit);
      a0 = av[0]; a1 = av[1]; a2 = av[2]; a3 = av[3];
      p0 = pv[0]; p1 = pv[1]; p2 = pv[2]; p3 = pv[3];
    }
    const uint32_t cls = FULL ? 0u : ((p0 >> 1) & 1u);
    const uint32_t uE = addmod(addmod(x2, p2, M), p0 ? M - p0 : 0u, M);
    const uint32_t uO = addmod(addmod(x2, p3, M), p1 ? M - p1 : 0u, M);
    const uint32_t vf = addmod(addmod(x, p1, M), p0 ? M - p0 : 0u, M);
    // Every index below stays under 2M, the table's two periods, whatever the
    // marker values (a_r <= M, folded bases and offsets < M), so no clamps are
    // needed.  Any vanishing
    // sub-polynomial, E or O value sends the wave through the zero-safe
    // recomputation, which keeps the common path free of selects.
    const bool rare = (a0 == M) | (a1 == M) | (a2 == M) | (a3 == M);
    const uint32_t FE = fold(K2 - a0, M), FO = fold(K3 - a1, M);    // [0, M)
    // the bases a2 + FE, a3 + FO folded once each ([0, M)), so that the two
    // reads of each (offsets uE, uE + h below M) need no fold of their own
    const uint32_t bE = fold(a2 + FE, M), bO = fold(a3 + FO, M);
    const uint32_t Ep = tab_c<TM>(tab, gtab, M, bE + uE);
    const uint32_t Em = tab_c<TM>(tab, gtab, M, bE + addmod(uE, h, M));
    const uint32_t Op = tab_c<TM>(tab, gtab, M, bO + uO);
    const uint32_t Om = tab_c<TM>(tab, gtab, M, bO + addmod(uO, h, M));
    uint32_t zs = 0, odd;
    if (!__ballot(rare | (Ep == M) | (Em == M) | (Op == M) | (Om == M))) {
      const uint32_t G = fold(fold(a1 + K1 - a0, M), M) + M;       // [M, 2M)
      // O + F for the points x, -x (s even) and ix, -ix (s odd), folded once
      const uint32_t OFp = fold(Op + fold(G - Ep, M), M), OFm = fold(Om + fold(G - Em, M), M);
      uint32_t u = 0;
      uint32_t r[4];
      bool anyz = false;
#pragma unroll
      for (uint32_t s = 0; s < 4; ++s) {
        const uint32_t E = (s & 1u) ? Em : Ep;
        const uint32_t OF = (s & 1u) ? OFm : OFp;
        r[s] = tab_c<TM>(tab, gtab, M, OF + addmod(vf, s * step, M));
        u += ((E ^ r[s]) >> 1) & 1u;
        anyz |= r[s] == M;
      }
      if (__ballot(anyz)) {
        u = 0;
#pragma unroll
        for (uint32_t s = 0; s < 4; ++s) {
          const uint32_t E = (s & 1u) ? Em : Ep;
          const bool z = r[s] == M;
          zs += z;
          u += z ? 0u : (((E ^ r[s]) >> 1) & 1u);
        }
      }
      odd = (((a0 >> 1) ^ fix) & 1u) ? (4 - zs) - u : u;
    } else {
      const uint32_t v0 = zmul_c(a0, addmod(K.ll[0], p0, M), M);
      const uint32_t v1 = zmul_c(a1, addmod(K.ll[1], p1, M), M);
      const uint32_t v2 = zmul_c(a2, addmod(K.ll[2], p2, M), M);
      const uint32_t v3 = zmul_c(a3, addmod(K.ll[3], p3, M), M);
      const uint32_t ep = zadd_c<TM>(tab, gtab, M, v0, zmul_c(v2, x2, M));
      const uint32_t em = zadd_c<TM>(tab, gtab, M, v0, zmul_c(v2, addmod(x2, h, M), M));
      const uint32_t op = zadd_c<TM>(tab, gtab, M, v1, zmul_c(v3, x2, M));
      const uint32_t om = zadd_c<TM>(tab, gtab, M, v1, zmul_c(v3, addmod(x2, h, M), M));
      odd = 0;
#pragma unroll
      for (uint32_t s = 0; s < 4; ++s) {
        const uint32_t E = (s & 1u) ? em : ep;
        const uint32_t O = (s & 1u) ? om : op;
        const uint32_t f = zadd_c<TM>(tab, gtab, M, E, zmul_c(O, addmod(x, s * step, M), M));
        const bool z = f == M;
        zs += z;
        odd += z ? 0u : (((f >> 1) ^ K.blane ^ cls) & 1u);
      }
    }
    c.add_n(cls, 4, zs, odd);
  }
}

// Split over mu_2 = {1, -1} on a form C/D level (every odd q; used where 4
// does not divide q - 1): f(x) = E(x^2) + x O(x^2), so the points x and -x
// share the two sub-polynomial values at Y = x^2 and take one Zech addition
// each, f(+-x) = E (1 + (+-x) O / E).  Byte units as sweep_split_c; a
// vanishing E or O sends the wave through the zero-safe addition on
// absolute logs, a vanishing point value is recounted exactly.
template <int NC, bool FULL, int D, int TM>
__device__ __forceinline__ void sweep_split2_c(const LevelDesc& L, const uint32_t (&sdel_e)[NC], uint32_t d,
                                               uint32_t mask, const SplitConst& Ke, LevelCounts& c) {
  uint32_t sdel[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) sdel[i] = 2 * sdel_e[i];
  SplitConst K = Ke;
  K.ll[0] = 2 * Ke.ll[0];
  K.ll[1] = 2 * Ke.ll[1];
  const uint32_t M = 2 * L.M, tab = L.tab_off, h = M / 2;
  const uint32_t* gtab = L.gtab;
  const uint32_t K1 = M + submod(K.ll[1], K.ll[0], M);             // [M, 2M)
  const uint32_t fix = ((K.ll[0] >> 1) ^ K.blane) & 1u;
  const uint32_t sup = mask | (1u << d);
  const uint32_t nt = L.nt;
  const uint32_t* xt = L.xs_t;
  uint32_t xnext = (xt && nt) ? sload(xt, 0) : 0u;
  for (uint32_t it = 0; it < nt; ++it) {
    const uint32_t x = 2 * xnext;
    if (it + 1 < nt) xnext = xt ? sload(xt, it + 1) : it + 1;
    const uint32_t Y = addmod(x, x, M);
    uint32_t p0, p1, a0, a1;
    bool hit = false;
    if (FULL) {
      a0 = horner_class_c<NC, 2, 0, FULL, D, false, TM>(tab, gtab, sdel, M, d, sup, Y, p0, hit);
      a1 = horner_class_c<NC, 2, 1, FULL, D, false, TM>(tab, gtab, sdel, M, d, sup, Y, p1, hit);
      if (__ballot(hit)) {
        a0 = horner_class_c<NC, 2, 0, FULL, D, true, TM>(tab, gtab, sdel, M, d, sup, Y, p0, hit);
        a1 = horner_class_c<NC, 2, 1, FULL, D, true, TM>(tab, gtab, sdel, M, d, sup, Y, p1, hit);
      }
    } else {
      uint32_t av[4], pv[4];
      horner_classes_c<NC, 2, false, TM>(tab, gtab, sdel, M, d, sup, Y, av, pv, hit);
      if (__ballot(hit)) horner_classes_c<NC, 2, true, TM>(tab, gtab, sdel, M, d, sup, Y, av, pv, hit);
      a0 = av[0]; a1 = av[1];
      p0 = pv[0]; p1 = pv[1];
    }
    const uint32_t cls = FULL ? 0u : ((p0 >> 1) & 1u);
    // log(x O / E) relative to the class logs: x + t_1 Y - t_0 Y
    const uint32_t vf = addmod(addmod(x, p1, M), p0 ? M - p0 : 0u, M);
    uint32_t zs = 0, odd;
    if (!__ballot((a0 == M) | (a1 == M))) {
      // a1 < M and F1 < M: the base a1 + F1 folded once ([0, M)), so that
      // both reads (offsets below M) stay under 2M with no fold of their own
      const uint32_t F1 = fold(K1 - a0, M);                            // [0, M)
      const uint32_t b1 = fold(a1 + F1, M);
      const uint32_t rp = tab_c<TM>(tab, gtab, M, b1 + vf);
      const uint32_t rm = tab_c<TM>(tab, gtab, M, b1 + addmod(vf, h, M));
      uint32_t u = ((rp >> 1) & 1u) + ((rm >> 1) & 1u);
      if (__ballot((rp == M) | (rm == M))) {
        zs = (rp == M) + (rm == M);
        u = (rp == M ? 0u : ((rp >> 1) & 1u)) + (rm == M ? 0u : ((rm >> 1) & 1u));
      }
      odd = (((a0 >> 1) ^ fix) & 1u) ? (2 - zs) - u : u;
    } else {
      const uint32_t v0 = zmul_c(a0, addmod(K.ll[0], p0, M), M);
      const uint32_t v1 = zmul_c(a1, addmod(K.ll[1], p1, M), M);
      odd = 0;
#pragma unroll
      for (uint32_t s = 0; s < 2; ++s) {
        const uint32_t f = zadd_c<TM>(tab, gtab, M, v0, zmul_c(v1, addmod(x, s * h, M), M));
        const bool z = f == M;
        zs += z;
        odd += z ? 0u : (((f >> 1) ^ K.blane ^ cls) & 1u);
      }
    }
    c.add_n(cls, 2, zs, odd);
  }
}

// Counts for one level: returns z | ns << 8 (roots and non-squares among the
// swept x; squares are nx - z - ns).  plog > 0: only part `part` of 2^plog
// consecutive shares of the level's point lists (the counts of the parts add
// up to the level's); where a list is implicit (full sweep), part 0 sweeps
// the whole level and the other parts nothing.
template <int G>
__device__ __forceinline__ uint32_t count_level(const LevelDesc& Lp, uint32_t lb, const uint32_t (&code)[2 * G + 3],
                                uint32_t top, uint32_t mask, uint32_t part = 0, uint32_t plog = 0) {
  constexpr int NC = 2 * G + 3;
  // the level with its table offsets made absolute LDS addresses
  LevelDesc L = Lp;
  L.tab_off += lb;
  L.emb_off += lb;
  const uint32_t M = L.M;
  const uint32_t d = top ? NC - 1 : NC - 2;
  uint32_t lc[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    // nonzero codes have logs below M; only a rejected row can reach M here
    const uint32_t v = lds_u32(L.emb_off + 4 * code[i]);
    lc[i] = v < M ? v : M - 1;
  }
  uint32_t prev = top ? lc[NC - 1] : lc[NC - 2];
  uint32_t del[NC];
#pragma unroll
  for (int i = NC - 2; i >= 0; --i) {
    del[i] = 0;
    if ((uint32_t)i < d && ((mask >> i) & 1u)) {
      uint32_t v = prev + M - lc[i];
      v = v >= M ? v - M : v;
      del[i] = v;
      prev = lc[i];
    }
  }
  del[NC - 1] = 0;
  const uint32_t blane = prev & 1u;  // parity of log c_low
  LevelCounts c = {0, 0, 0, 0, 0};
  const bool full = mask == ((1u << d) - 1u);
  // split evaluation: needs every class to hold a term (forms C/D: m = 4)
  const uint32_t sup = mask | (1u << d);
  uint32_t ms = L.msplit;
  if (L.form != kFormA && ms != 4 && ms != 2) ms = 0;
  if (ms) {
    uint32_t cls_mask = 0;
#pragma unroll
    for (int i = 0; i < NC; ++i)
      if ((sup >> i) & 1u) cls_mask |= 1u << (ms == 4 ? i % 4 : (ms == 3 ? i % 3 : i % 2));
    if (cls_mask != (1u << ms) - 1u) ms = 0;
  }
  if (plog) {
    if (ms ? (L.xs_t != nullptr && L.xs_s != nullptr) : (L.xs != nullptr)) {
      if (ms) {
        const uint32_t t0 = (L.nt * part) >> plog, t1 = (L.nt * (part + 1)) >> plog;
        const uint32_t s0 = (L.ns * part) >> plog, s1 = (L.ns * (part + 1)) >> plog;
        L.xs_t += t0;
        L.nt = t1 - t0;
        L.xs_s += s0;
        L.ns = s1 - s0;
        L.nx = L.nt * ms + L.ns;
      } else {
        const uint32_t x0 = (L.nx * part) >> plog, x1 = (L.nx * (part + 1)) >> plog;
        L.xs += x0;
        L.nx = x1 - x0;
      }
    } else if (part) {
      L.nx = L.nt = L.ns = 0;
    }
  }
  // per-class relative deltas (element units) and lowest-coefficient logs
  uint32_t sdel[NC];
  SplitConst K;
  K.ll[0] = K.ll[1] = K.ll[2] = K.ll[3] = 0;
  K.blane = blane;
#pragma unroll
  for (int i = 0; i < NC; ++i) sdel[i] = 0;
  if (ms) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (r >= (int)ms) break;
      bool started = false;
      uint32_t pv = 0;
#pragma unroll
      for (int i = NC - 1; i >= 0; --i) {
        const uint32_t cl = ms == 4 ? (uint32_t)(i % 4) : (ms == 3 ? (uint32_t)(i % 3) : (uint32_t)(i % 2));
        if (cl != (uint32_t)r || (uint32_t)i > d || !((sup >> i) & 1u)) continue;
        if (started) {
          uint32_t v = pv + M - lc[i];
          v = v >= M ? v - M : v;
          sdel[i] = v;
        }
        started = true;
        pv = lc[i];
      }
      K.ll[r] = pv;
    }
  }
  if (L.form == kFormA) {
    // byte units plus the table offset
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      del[i] = 2 * del[i] + L.tab_off;
      sdel[i] = 2 * sdel[i] + L.tab_off;
    }
    if (ms) {
#define HWC_SPLIT(FULLV, DV)                                                         \
  do {                                                                               \
    if (ms == 4) sweep_split_a<NC, 4, FULLV, DV>(L, sdel, del, d, mask, K, c);      \
    else if (ms == 3) sweep_split_a<NC, 3, FULLV, DV>(L, sdel, del, d, mask, K, c); \
    else sweep_split_a<NC, 2, FULLV, DV>(L, sdel, del, d, mask, K, c);              \
    sweep_form_a<NC, FULLV, DV>(L.xs_s, L.ns, M, del, d, mask, c);                  \
  } while (0)
      if (full) {
        if (top) HWC_SPLIT(true, NC - 1);
        else HWC_SPLIT(true, NC - 2);
      } else {
        HWC_SPLIT(false, 0);
      }
#undef HWC_SPLIT
    } else {
      if (full) {
        if (top) sweep_form_a<NC, true, NC - 1>(L.xs, L.nx, M, del, d, mask, c);
        else sweep_form_a<NC, true, NC - 2>(L.xs, L.nx, M, del, d, mask, c);
      } else {
        sweep_form_a<NC, false, 0>(L.xs, L.nx, M, del, d, mask, c);
      }
    }
  } else {
    // byte units; a form C, E, F or G table starts the LDS image
    L.tab_off = lb;
#define HWC_FORM_C(GL)                                                                   \
  do {                                                                                   \
    if (ms == 4) {                                                                       \
      if (full) {                                                                        \
        if (top) sweep_split_c<NC, true, NC - 1, GL>(L, sdel, d, mask, K, c);            \
        else sweep_split_c<NC, true, NC - 2, GL>(L, sdel, d, mask, K, c);                \
      } else {                                                                           \
        sweep_split_c<NC, false, 0, GL>(L, sdel, d, mask, K, c);                         \
      }                                                                                  \
      sweep_form_c<NC, GL>(L, L.xs_s, L.ns, del, d, mask, c);                            \
    } else if (ms == 2) {                                                                \
      if (full) {                                                                        \
        if (top) sweep_split2_c<NC, true, NC - 1, GL>(L, sdel, d, mask, K, c);           \
        else sweep_split2_c<NC, true, NC - 2, GL>(L, sdel, d, mask, K, c);               \
      } else {                                                                           \
        sweep_split2_c<NC, false, 0, GL>(L, sdel, d, mask, K, c);                        \
      }                                                                                  \
      sweep_form_c<NC, GL>(L, L.xs_s, L.ns, del, d, mask, c);                            \
    } else {                                                                             \
      sweep_form_c<NC, GL>(L, L.xs, L.nx, del, d, mask, c);                              \
    }                                                                                    \
  } while (0)
    if (L.form == kFormC) HWC_FORM_C(kTabC);
    else if (L.form == kFormE) HWC_FORM_C(kTabE);
    else if (L.form == kFormF) HWC_FORM_C(kTabF);
    else if (L.form == kFormG) HWC_FORM_C(kTabG);
    else HWC_FORM_C(kTabD);
#undef HWC_FORM_C
  }
  const uint32_t n0 = L.nx - c.n1;
  const uint32_t z = c.zt;
  const uint32_t z0 = c.zt - c.z1, o0 = c.ot - c.o1;
  // chi(f(x)) = (-1)^(A + log c_low + low*L); A odd counted in o*, zeros are even
  const uint32_t ns0 = blane ? (n0 - z0 - o0) : o0;
  const uint32_t ns1 = blane ? c.o1 : (c.n1 - c.z1 - c.o1);
  return z | ((ns0 + ns1) << 8);
}

// N_k from the per-level counts (Sec. 1.1 decomposition; x = 0 and the
// points at infinity of the model in P(1, g+1, 1) added here).
template <int G>
__device__ __forceinline__ void assemble(const PlanDesc& P, const uint32_t (&lv)[G], uint32_t c0, uint32_t ctop,
                                         uint32_t log0, uint32_t logtop, int32_t* out) {
#pragma unroll
  for (int k = 1; k <= G; ++k) {
    const int chi0 = (k % 2 == 0) ? 1 : ((log0 & 1u) ? -1 : 1);
    const int chit = (k % 2 == 0) ? 1 : ((logtop & 1u) ? -1 : 1);
    int32_t n = (c0 == 0 ? 1 : 1 + chi0) + (ctop == 0 ? 1 : 1 + chit);
    if (P.orbit) {
#pragma unroll
      for (int j = 1; j <= G; ++j) {
        if (k % j) continue;
        const uint32_t z = lv[j - 1] & 0xFFu, ns = lv[j - 1] >> 8;
        const uint32_t s = P.lv[j - 1].nx - z - ns;
        const uint32_t sq = ((k / j) % 2 == 0) ? s + ns : s;
        n += (int32_t)(j * z + 2 * j * sq);
      }
    } else {
      const uint32_t z = lv[k - 1] & 0xFFu, ns = lv[k - 1] >> 8;
      const uint32_t s = P.lv[k - 1].nx - z - ns;
      n += (int32_t)(z + 2 * s);
    }
    out[k - 1] = n;
  }
}

// One tile (up to 64 curves of one pattern) through levels lvl_lo..lvl_hi.
// With plog > 0 this is part `part` of tile `tile`: the levels below the top
// belong to part 0, the top level's points are shared out (count_level); the
// part adds its counts into acc, and the tile's last part to finish reads the
// sums back and assembles N.
template <int G, typename CT>
__device__ __forceinline__ void process_tile(const PlanDesc& P, uint32_t lb, const CT* __restrict__ codes,
                                             const uint32_t* __restrict__ perm, uint64_t w, uint32_t lvl_lo,
                                             uint32_t lvl_hi, int32_t* __restrict__ outN,
                                             uint32_t* __restrict__ outLv, uint32_t tile = 0, uint32_t part = 0,
                                             uint32_t plog = 0, uint32_t* __restrict__ acc = nullptr,
                                             uint32_t* __restrict__ done = nullptr) {
  constexpr int NC = 2 * G + 3;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t pat = uniform((uint32_t)(w & 0xFFFFu));
  const uint32_t cnt = uniform((uint32_t)((w >> 16) & 0xFFFFu) + 1u);
  const uint32_t start = uniform((uint32_t)(w >> 32));
  // every lane runs the tile so that pattern branches stay uniform; lanes past
  // the tile's end shadow its last curve and skip the stores
  const bool live = lane < cnt;
  const uint32_t curve = perm[start + (live ? lane : cnt - 1)];
  uint32_t code[NC];
  const CT* row = codes + (uint64_t)curve * NC;
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    int v = (int)row[i];
    v = v < 0 ? 0 : (v >= (int)P.q ? (int)P.q - 1 : v);  // keeps reads in bounds on bad input
    code[i] = (uint32_t)v;
  }
  const uint32_t top = (pat >> (NC - 1)) & 1u;
  const uint32_t mask = pat & ((1u << (NC - 1)) - 1u);
  // levels one after another (one inlined copy of the level code); the
  // level descriptor comes in through scalar loads
  uint32_t lv[G];
#pragma unroll
  for (int j = 0; j < G; ++j) lv[j] = 0;
#pragma unroll 1
  for (uint32_t j = lvl_lo; j <= lvl_hi; ++j) {
    const bool shared = j + 1 == (uint32_t)G;
    if (part && !shared) continue;
    const uint32_t v = count_level<G>(load_level(P, j), lb, code, top, mask, shared ? part : 0u, shared ? plog : 0u);
#pragma unroll
    for (int k = 0; k < G; ++k) lv[k] = (uint32_t)k == j ? v : lv[k];
  }
  if (plog) {
    // packed counts add without carries: a level's zeros stay below 256
    if (live) {
#pragma unroll
      for (int k = 0; k < G; ++k)
        if (lv[k]) atomicAdd(acc + (uint64_t)curve * G + k, lv[k]);
    }
    __threadfence();
    uint32_t prior = 0;
    if (lane == 0) prior = atomicAdd(done + tile, 1u);
    if (uniform(prior) != (1u << plog) - 1u) return;
    __threadfence();
#pragma unroll
    for (int k = 0; k < G; ++k)
      lv[k] = __hip_atomic_load(acc + (uint64_t)curve * G + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }

  if (outN) {
    const uint32_t log0 = lds_u32(lb + P.lv[0].emb_off + 4 * code[0]);
    const uint32_t logt = lds_u32(lb + P.lv[0].emb_off + 4 * code[NC - 1]);
    int32_t n[G];
    assemble<G>(P, lv, code[0], code[NC - 1], log0, logt, n);
    if (live) {
#pragma unroll
      for (int k = 0; k < G; ++k) outN[(uint64_t)curve * G + k] = n[k];
    }
  }
  if (outLv && live) {
#pragma unroll
    for (int j = 0; j < G; ++j)
      if ((uint32_t)j >= lvl_lo && (uint32_t)j <= lvl_hi) outLv[(uint64_t)curve * G + j] = lv[j];
  }
}

// WPE: minimum waves per SIMD the register allocation must allow (1: free)
template <int G, typename CT, int WPE>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(WPE))) void count_kernel(const PlanDesc* __restrict__ Pd, const CT* __restrict__ codes,
                                                     const uint32_t* __restrict__ perm,
                                                     const uint64_t* __restrict__ tiles,
                                                     const uint32_t* __restrict__ ntiles_p, uint32_t* queue,
                                                     uint32_t lvl_lo, uint32_t lvl_hi, int32_t* __restrict__ outN,
                                                     uint32_t* __restrict__ outLv, uint32_t plog,
                                                     uint32_t* __restrict__ acc, uint32_t* __restrict__ done) {
  const PlanDesc& P = *Pd;
  extern __shared__ uint32_t lds32[];
  constexpr uint32_t lb = kImageBase;
  for (uint32_t i = threadIdx.x; i < P.image_bytes / 4; i += blockDim.x) lds32[i] = P.image[i];
  __syncthreads();
  const uint32_t lane = threadIdx.x & (kWave - 1);
  // queue entries: tiles, or (plog > 0, levels 0..G-1 through the queue) the
  // 2^plog parts of every tile, as in the batch kernel
  const uint32_t ntiles = *ntiles_p << plog;
  const uint32_t pmask = (1u << plog) - 1u;
  const uint32_t nwaves = (gridDim.x * blockDim.x) / kWave;
  uint32_t t;
  if (queue) {
    uint32_t v = 0;
    if (lane == 0) v = atomicAdd(queue, 1u);
    t = uniform(v);
  } else {
    t = uniform((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  }
  while (t < ntiles) {
    process_tile<G, CT>(P, lb, codes, perm, sload64(tiles, t >> plog), lvl_lo, lvl_hi, outN, outLv, t >> plog,
                        t & pmask, plog, acc, done);
    if (queue) {
      uint32_t v = 0;
      if (lane == 0) v = atomicAdd(queue, 1u);
      t = uniform(v);
    } else {
      t = uniform(t + nwaves);
    }
  }
}

// ----------------------------------------------------------------------------
// one persistent launch over several plans: waves pop the tiles of one job
// at a time; a workgroup restages LDS when the job's plan differs from the
// staged one.

// GMAX: the largest genus of the batch; the kernel holds the tile code of
// every genus up to it only, so its register budget (and with it the waves a
// CU keeps in flight, which latency-bound device-memory tables need) is that
// of the batch's genera, not of g = 4.
template <int GMAX>
__device__ __forceinline__ void process_job_tile(const JobDesc& J, uint32_t lb, uint32_t u) {
  const PlanDesc& P = *J.plan;
  const uint32_t plog = J.plog, tile = u >> plog, part = u & ((1u << plog) - 1u);
  const uint64_t w = sload64(J.tiles, tile);
#define HWC_JOB(GG)                                                                                      \
  case GG:                                                                                               \
    if constexpr (GG <= GMAX) {                                                                          \
      if (J.cb == 1)                                                                                     \
        process_tile<GG, int8_t>(P, lb, static_cast<const int8_t*>(J.codes), J.perm, w, 0, GG - 1, J.outN, \
                                 nullptr, tile, part, plog, J.acc, J.done);                              \
      else                                                                                               \
        process_tile<GG, int16_t>(P, lb, static_cast<const int16_t*>(J.codes), J.perm, w, 0, GG - 1,     \
                                  J.outN, nullptr, tile, part, plog, J.acc, J.done);                     \
    }                                                                                                    \
    break;
  switch (J.g) {
    HWC_JOB(1) HWC_JOB(2) HWC_JOB(3) HWC_JOB(4)
    default: break;
  }
#undef HWC_JOB
}

// One persistent launch over the jobs of a batch, taken in the order given
// (most expensive tiles first).  Every wave pops tiles of the current job from
// the job's own queue and moves to the next job when that queue is empty; a
// workgroup restages its LDS image only when the next job that still has
// tiles uses another plan, and only there waits at barriers.  slot: byte
// offset, past every image, of the word that broadcasts whether a job still
// has tiles (inside the dynamic block, so the kernel has no static LDS).
template <int GMAX>
__global__ __launch_bounds__(1024) void batch_kernel(const JobDesc* __restrict__ jobs, uint32_t njobs,
                                                     uint32_t slot) {
  extern __shared__ uint32_t lds32[];
  uint32_t& sh_open = *reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(lds32) + slot);
  constexpr uint32_t lb = kImageBase;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const PlanDesc* staged = nullptr;
  for (uint32_t k = 0; k < njobs; ++k) {
    const JobDesc& J = jobs[k];
    const uint32_t nt = *J.ntiles << J.plog;   // queue entries: tiles, or parts of tiles
    const PlanDesc* P = J.plan;
    if (P != staged) {
      __syncthreads();   // every wave is done with the image staged so far
      if (threadIdx.x == 0) sh_open = atomicAdd(J.queue, 0u) < nt ? 1u : 0u;
      __syncthreads();
      if (!sh_open) continue;   // nothing left here: no restaging
      const uint32_t* img = P->image;
      const uint32_t nwords = P->image_bytes / 4;
      for (uint32_t w = threadIdx.x; w < nwords; w += blockDim.x) lds32[w] = img[w];
      __syncthreads();
      staged = P;
    }
    for (;;) {
      uint32_t v = 0;
      if (lane == 0) v = atomicAdd(J.queue, 1u);
      const uint32_t t = uniform(v);
      if (t >= nt) break;
      process_job_tile<GMAX>(J, lb, t);
    }
  }
}

}  // namespace hwc
