// Device-side description of one (q, g) counting plan, shared by the HIP
// kernels and the host code that builds it.
//
// A plan covers the fields F_{q^j}, j = 1..g (one "level" per field).  All
// of its lookup tables are packed into one image that every workgroup copies
// into LDS before it starts counting:
//
//   form A  (M <= 10922)  "byte units":  5M u16 entries.  Entry i < 3M holds
//           2*Z(i mod M), or the zero marker 6M when 1 + gamma^(i mod M) = 0;
//           entries 3M..5M-1 hold 0.  One Horner step is one add and one read.
//   form C  (M <= 32767)  "element units": 2M u16 entries.  Entry i holds
//           Z(i mod M), or M as the zero marker.  One Horner step is add,
//           fold into [0, 2M), scale to bytes, read, and a marker test.
//   form E  (M <= 65534)  "element units, one period": M u16 entries, entry
//           i holds Z(i), or M as the zero marker.  A step folds its index
//           into the period once more than form C and doubles the entry it
//           reads, so it shares form C's code; twice the field size of form C
//           fits in LDS.
//   form F  (M <= 131070)  "half table": Z(k) for k = 0..M/2 only, as u16
//           low halves followed by a bitmap of the 17th bits; the other half
//           follows from Z(-k) = Z(k) - k (1 + g^-k = g^-k (1 + g^k)), so
//           Z(k) = Z(M - k) + k mod M for k > M/2.  Two reads per lookup.
//   form D  (any M)  the form C layout with u32 entries, kept in device
//           memory (L2/MALL-resident) when the level does not fit in LDS.
//   emb     q u32 entries: log of the F_q code c in F_{q^j}, or M for c = 0.
//
// Logs are taken to the primitive element gamma of each F_{q^j}; Z is the
// Zech logarithm Z(k) = log(1 + gamma^k) (eq. 2.1, table (3.2)).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hwc {

constexpr int kMaxG = 4;                 // genus handled by the kernels
constexpr int kMaxCoef = 2 * kMaxG + 3;  // a_0 .. a_{2g+2}
constexpr uint32_t kFormA = 0, kFormC = 1, kFormD = 2, kFormE = 3, kFormF = 4, kFormG = 5;
constexpr uint32_t kFormAMaxM = 10922;   // 6M must fit in u16
constexpr uint32_t kFormCMaxM = 32767;   // M must fit in 15 bits
constexpr uint32_t kFormEMaxM = 65534;   // M (the zero marker) must fit in u16
constexpr uint32_t kFormFMaxM = 131070;  // M must fit in 17 bits, M/2 + 1 entries in the half table
// Form G: the half table of form F as u32 entries in byte units (one read, no
// bit plane), used where its 4 (M/2 + 1) bytes fit the LDS image
constexpr int kWave = 64;
// LDS of one CU is 160 KiB; 256 bytes stay free for the kernels' own variables
constexpr uint32_t kLdsImageLimit = 160 * 1024 - 256;
// Dense translates (rows replaced by f(x + t), see shift_kernel): fields with
// q <= kShiftMaxQ, whose q^3-byte step table fits LDS, at most kShiftTries t.
constexpr uint32_t kShiftMaxQ = 32;
constexpr uint32_t kShiftTries = 8;
// For prime q the translate is also an integer matrix product: after the
// step table (q^3 bytes, padded to 16) the shift buffer holds, for t = 0 ..
// kShiftTries, the rows i = 0 .. NC-2 of binom(j, i) t^(j-i) mod q (j >= i,
// zero below), bytes packed four to a word: shift_tmat_words(NC) words per t.
inline constexpr uint32_t shift_tmat_offset_words(uint32_t q) { return (q * q * q + 15) / 16 * 4; }
inline constexpr uint32_t shift_tmat_row_words(uint32_t nc) { return (nc + 3) / 4; }
inline constexpr uint32_t shift_tmat_words(uint32_t nc) { return (nc - 1) * shift_tmat_row_words(nc); }

struct LevelDesc {
  uint32_t M;         // |F_{q^j}^x|
  uint32_t form;      // kFormA, kFormC, kFormD, kFormE, kFormF or kFormG
  uint32_t tab_off;   // byte offset of the level's table in the image
  uint32_t emb_off;   // byte offset of the level's emb table in the image
  uint32_t nx;        // number of x logs swept at this level
  uint32_t weight;    // points of F_{q^j} each swept x stands for (orbit size, or 1)
  const uint32_t* xs; // x logs (device), nullptr: x runs over 0..M-1
  const uint32_t* gtab;  // form D: 2M entries in device memory
  // split evaluation over mu_m cosets (m = 4, 3 or 2; forms C/D: 4 or 2): nt tuple
  // representatives (points L + s M/m, s < m) and ns single points; together
  // they are the same nx points.  msplit = 0 turns it off.
  uint32_t msplit, nt, ns;
  const uint32_t* xs_t;  // nullptr: representatives 0..M/m-1 (full sweep)
  const uint32_t* xs_s;
};

struct PlanDesc {
  uint32_t q, p, g, ncoef;   // q = p^e; ncoef = 2g+3
  uint32_t orbit;         // 1: level j sweeps primitive Frobenius orbits of F_{q^j}
  uint32_t image_bytes;   // LDS image size (multiple of 16)
  const uint32_t* image;  // device copy of the image (dwords)
  LevelDesc lv[kMaxG];
};

// Factorization partition code (eq. 1.2): the multiplicity of part j
// (j = 1..10, i.e. 2g+2 <= 10) sits in bits [lam_shift(j), lam_shift(j) + w_j)
// with widths w = 4, 3, 2, 2, 2, 1, 1, 1, 1, 1 -- enough for every partition
// of 10 -- so a code fits in kLamBits bits.
constexpr uint32_t kLamBits = 18;
constexpr uint32_t kLamInvalid = 0xFFFFFFFFu;   // root counts inconsistent with a square-free row
__host__ __device__ constexpr uint32_t lam_shift(uint32_t j) {
  return j == 1 ? 0u : j == 2 ? 4u : j == 3 ? 7u : j == 4 ? 9u : j == 5 ? 11u : 7u + j;
}

// The partition codes a histogram column can hold for genus g: 0 (the mark of
// a row with a square factor) and the code of every partition of 2g+2, in
// ascending order, so a code's rank there is a dense digit (at most 43 values,
// p(10) = 42) that sorts like the code. Writes them to out (room for
// kLamCodesMax, or nullptr) and returns how many there are.
constexpr uint32_t kLamCodesMax = 48;
inline uint32_t lam_code_list(uint32_t g, uint32_t* out) {
  uint32_t buf[kLamCodesMax];
  uint32_t n = 0;
  buf[n++] = 0;
  // parts in non-increasing order: stack of (remaining degree, largest part, code)
  struct Frame { uint32_t rem, maxp, code; };
  Frame st[64];                          // pending siblings along one path: <= 10 + 9 + .. + 1
  uint32_t top = 0;
  st[top++] = {2 * g + 2, 2 * g + 2, 0};
  while (top) {
    const Frame f = st[--top];
    if (f.rem == 0) {
      if (n < kLamCodesMax) buf[n++] = f.code;
      continue;
    }
    for (uint32_t j = 1; j <= f.maxp && j <= f.rem; ++j) st[top++] = {f.rem - j, j, f.code + (1u << lam_shift(j))};
  }
  for (uint32_t i = 1; i < n; ++i)   // insertion sort (n <= 43)
    for (uint32_t k = i; k > 0 && buf[k - 1] > buf[k]; --k) {
      const uint32_t t = buf[k];
      buf[k] = buf[k - 1];
      buf[k - 1] = t;
    }
  if (out)
    for (uint32_t i = 0; i < n; ++i) out[i] = buf[i];
  return n;
}

// One curve for the lane-per-x kernel: coefficient logs in F_{q^k} (M where
// the coefficient is zero), degree d, M = q^k - 1.
struct SingleDesc {
  uint32_t lc[2 * kMaxG + 3];
  uint32_t d, M;
};

// Counting by F_p-linear algebra (prime q = p): with F_{p^j} = F_p[t]/(P) and
// x^i = sum_d a_{i,d} t^d, f(x) = sum_i c_i x^i has coordinates
// D_d = sum_i c_i a_{i,d} mod p, i.e. the codes times a Vandermonde matrix of
// coordinates -- an int8 matrix product for the matrix cores.  The image holds,
// per level, the swept points in blocks of 32 as the A operand of
// v_mfma_i32_32x32x16_i8 ([block][d][row][16 bytes]; coordinate 0 times 4, so
// its residue mod 4p is four times the residue mod p), then a u32 table of the
// quadratic character over packed elements (byte offset 4 sum_d r_d p^d):
// 0 square, 1 nonsquare, kVZero for zero.  Needs 4(p-1) <= 127: p <= 31.
// When a level's blocks do not fit one image, its points are split over
// several images (passes) that add their counts per curve; such a level may
// use a u16 table (byte offset 2 sum_d r_d p^d, coordinate 0 doubled).
// The K slots past the coefficients hold 127 on the curve side and, in the
// coordinate-0 rows, values summing to to / 127, so the product adds the
// table's byte offset (a multiple of 508) to coordinate 0 by itself.
constexpr uint32_t kVSlotUnit = 127;
constexpr uint32_t kVZero = 1u << 15;
constexpr uint32_t kVMaxP = 31;
struct VLevel {
  uint32_t pts, nblk;     // swept points in the image and their 32-point blocks
  uint32_t pad;           // padding rows of the blocks (zero points, subtracted)
  uint32_t vo, to;        // byte offsets of the blocks and of the character table
  uint32_t m0, s0;        // floor(v / 4p) = (v * m0) >> s0 for every value coordinate 0 reaches
  uint32_t nbm0;          // -to * m0 mod 2^32: coordinate 0 arrives with the table offset added
  uint32_t m1, s1;        // floor(v / p) = (v * m1) >> s1 for the other coordinates
};
// Balanced form (p = 11, 13): digits and coefficients in -(p-1)/2 .. (p-1)/2,
// coefficients times sb, coordinates d >= 1 times p, coordinate 0 times tw/sb,
// and constants in the spare K slots that make every value nonnegative and
// a multiple of the divisor where it must vanish; then coordinate d >= 1 is
// sb p D_d + 127 sb p^2 and its quotient by sb p^2 (>= 256) is one 24-bit
// multiply-high by m1.
struct VPlanDesc {
  uint32_t p, g, ncoef, orbit;
  uint32_t bal, sb;       // balanced form and the coefficient scale
  uint32_t image_bytes;
  const uint32_t* image;
  VLevel lv[kMaxG];
};

// One request of a multi-plan launch (device memory).
struct JobDesc {
  const PlanDesc* plan;   // device copy of the job's plan
  const void* codes;      // [n][2g+3] int8 or int16
  const uint32_t* perm;   // bucketed order of the job's rows
  const uint64_t* tiles;  // the job's tile words
  const uint32_t* ntiles; // number of tile words (written by the bucketing)
  uint32_t* queue;        // the job's tile queue (set to 0 by the bucketing)
  int32_t* outN;          // [n][g]
  uint32_t cb, g;         // code bytes, genus
  // The top level's sweep of every tile cut into 2^plog parts (queue entry
  // u: tile u >> plog, part u & (2^plog - 1)) when a job has few tiles for
  // the waves in flight: the parts add their level counts into acc and the
  // last part of a tile (counted in done) assembles N.  plog = 0: whole tiles.
  uint32_t plog;
  uint32_t* acc;          // [n][g] packed level counts (zero before the launch)
  uint32_t* done;         // [tiles] parts finished (zero before the launch)
};

// A tile is up to 64 curves that share degree and zero pattern.
// word = pattern | (count-1) << 16 | start << 32
__host__ __device__ inline uint64_t tile_pack(uint32_t pattern, uint32_t start, uint32_t count) {
  return (uint64_t)pattern | ((uint64_t)(count - 1) << 16) | ((uint64_t)start << 32);
}

// Pattern of a row: bit 2g+2 set when deg f = 2g+2; bits 0..d-1 mark the
// nonzero a_i below the leading term.
__host__ __device__ inline uint32_t pattern_count(uint32_t g) { return 1u << (2 * g + 3); }

}  // namespace hwc
