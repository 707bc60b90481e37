// Kernels around the count on gfx950: dense translates, bucketing by zero
// pattern, the assembly and partition kernels, the map's representatives, the
// one-curve sweep, and the host-callable launchers.  The count itself (the
// relative-log Horner sweeps and the persistent count and batch kernels) is
// in count_impl.h, built per genus in count_g1.hip .. count_g4.hip.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "count_entry.h"
#include "count_impl.h"
#include "plan.h"

namespace hwc {

// ----------------------------------------------------------------------------
// utility

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ----------------------------------------------------------------------------
// classification: validate rows, compute the pattern of each row and the
// number of rows per pattern.

// hist[pat] += 1 for every active lane, one LDS atomic per distinct pattern in
// the wave (rows of a wave mostly share one or two patterns, so per-lane
// atomics would serialize on the same address).
__device__ __forceinline__ void wave_count(uint32_t* hist, uint32_t pat, bool active) {
  uint64_t left = __ballot(active);
  while (left) {
    const uint32_t leader = uniform((uint32_t)__builtin_amdgcn_readlane((int)pat, (int)__builtin_ctzll(left)));
    const uint64_t same = __ballot(active && pat == leader);
    if ((threadIdx.x & (kWave - 1)) == (uint32_t)__builtin_ctzll(left)) atomicAdd(&hist[leader], (uint32_t)__popcll(same));
    left &= ~same;
  }
}

template <typename CT>
__global__ __launch_bounds__(256) void classify_kernel(const CT* __restrict__ codes, uint64_t n, uint32_t q,
                                                       uint32_t g, uint16_t* __restrict__ pid,
                                                       uint32_t* __restrict__ counts, uint32_t* __restrict__ err) {
  extern __shared__ uint32_t hist[];
  const uint32_t npat = pattern_count(g);
  const uint32_t nc = 2 * g + 3;
  for (uint32_t i = threadIdx.x; i < npat; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  uint32_t bad = 0;
  // every lane of a wave runs the same number of iterations (wave_count has ballots)
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t base = blockIdx.x * (uint64_t)blockDim.x + (threadIdx.x & ~(uint32_t)(kWave - 1));
  for (uint64_t w0 = base; w0 < n; w0 += stride) {
    const uint64_t i = w0 + (threadIdx.x & (kWave - 1));
    const bool live = i < n;
    uint32_t pat = 0;
    if (live) {
      const CT* row = codes + i * nc;
      uint32_t mask = 0;
      const int top = (int)row[nc - 1], sub = (int)row[nc - 2];
      const uint32_t d = top ? nc - 1 : nc - 2;
      for (uint32_t j = 0; j < nc; ++j) {
        const int c = (int)row[j];
        if (c < 0 || c >= (int)q) bad |= 1u;
        if (j < d && c != 0) mask |= 1u << j;
      }
      if (top == 0 && sub == 0) bad |= 2u;
      pat = (top ? (1u << (nc - 1)) : 0u) | mask;
      pid[i] = (uint16_t)pat;
    }
    wave_count(hist, pat, live);
  }
  if (bad) atomicOr(err, bad);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < npat; i += blockDim.x)
    if (hist[i]) atomicAdd(&counts[i], hist[i]);
}

// Dense translates.  x -> x + t (t in F_q) permutes every F_{q^k} and keeps
// the degree and the leading coefficient, so f(x + t) has the same N_k, the
// same factorization pattern and the same discriminant as f (the same
// equivalence the reduced enumeration of Algorithm 1 divides out).  A row with
// a zero coefficient below its leading one is replaced by f(x + t) for the
// first code t = 1, 2, .. (at most kShiftTries of them) that leaves no such
// zero; a row without one, or with codes out of range, is copied as it is.
// Dense rows take the counting kernels' straight-line path, which is cheaper
// than the sparse one even though it has more terms.
//
// The coefficients of f(x + t) come from repeated synthetic division: for
// k = 0 .. D-1 and i = D-1 down to k, w_i <- w_i + t w_{i+1}.  Each step is one
// read of the LDS table step[t][a][b] = a + t b (F_q codes, q^3 bytes); fully
// unrolled, the steps' dependences form a triangle whose longest chain is 2D.
//
// DOT (prime q): the coefficients of f(x + t) are v_i = sum_{j >= i}
// binom(j, i) t^(j-i) c_j mod q, an integer matrix product done with 4-byte
// dot products (the matrix rows of each t come packed after the step table,
// see shift_tmat_offset_words); the sums stay below NC (q-1)^2 < 2^14, and
// v mod q = v - q floor(v qm / 2^20) with qm = ceil(2^20 / q) is exact for
// v < 2^20 / q.  No LDS reads: the vector ALU does what the table did.
//
// With pid given, the kernel also classifies the rows it writes, as
// classify_kernel does (pattern per row, rows per pattern added to counts,
// error bits), so the bucketing needs no second pass over them.
template <int NC, typename CT, bool DOT>
__global__ __launch_bounds__(256) void shift_kernel(const CT* __restrict__ in, uint64_t n, uint32_t q,
                                                    const uint32_t* __restrict__ step, CT* __restrict__ out,
                                                    uint16_t* __restrict__ pid, uint32_t* __restrict__ counts,
                                                    uint32_t* __restrict__ err, uint32_t qm) {
  extern __shared__ uint32_t sh32[];
  constexpr uint32_t npat = 1u << NC;
  constexpr uint32_t NW = shift_tmat_row_words(NC);
  const uint32_t qq = q * q, words = DOT ? 0u : (qq * q + 3) / 4;
  uint32_t* hist = sh32 + (words + 3) / 4 * 4;     // after the step table
  for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) sh32[i] = step[i];
  const uint32_t* __restrict__ tmat = step + shift_tmat_offset_words(q);
  if (pid)
    for (uint32_t i = threadIdx.x; i < npat; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  const uint8_t* tab = reinterpret_cast<const uint8_t*>(sh32);
  uint32_t bad = 0;
  // every lane of a wave runs the same number of iterations (ballots below)
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t base = blockIdx.x * (uint64_t)blockDim.x + (threadIdx.x & ~(uint32_t)(kWave - 1));
  for (uint64_t w0 = base; w0 < n; w0 += stride) {
    const uint64_t r = w0 + (threadIdx.x & (kWave - 1));
    const bool live = r < n;
    CT raw[NC];
    uint32_t c[NC];
    bool valid = live;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      raw[i] = live ? in[r * NC + i] : (CT)0;
      const int v = (int)raw[i];
      valid = valid && v >= 0 && v < (int)q;
      c[i] = (v >= 0 && v < (int)q) ? (uint32_t)v : 0u;
    }
    const uint32_t d = c[NC - 1] ? NC - 1 : NC - 2;
    bool need = false;
#pragma unroll
    for (int i = 0; i < NC - 1; ++i) need = need || ((uint32_t)i < d && c[i] == 0);
    need = need && valid && c[d] != 0;
    bool done = false;
    uint32_t w[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) w[i] = c[i];
    uint32_t cp[NW];
    if constexpr (DOT) {
#pragma unroll
      for (uint32_t w = 0; w < NW; ++w) {
        uint32_t word = 0;
#pragma unroll
        for (uint32_t b = 0; b < 4; ++b)
          if (4 * w + b < (uint32_t)NC) word |= c[4 * w + b] << (8 * b);
        cp[w] = word;
      }
    }
    for (uint32_t t = 1; t < q && t <= kShiftTries; ++t) {
      if (!__ballot(need && !done)) break;
      uint32_t v[NC];
      if constexpr (DOT) {
        const uint32_t* Tt = tmat + t * shift_tmat_words(NC);
#pragma unroll
        for (int i = 0; i < NC - 1; ++i) {
          uint32_t acc = 0;
#pragma unroll
          for (uint32_t w = (uint32_t)i / 4; w < NW; ++w)
            acc = __builtin_amdgcn_udot4(Tt[i * NW + w], cp[w], acc, false);
          v[i] = acc - __umul24(q, __umul24(acc, qm) >> 20);   // 24-bit products, full rate
        }
        v[NC - 1] = c[NC - 1];
      } else {
        const uint32_t base = t * qq;
#pragma unroll
        for (int i = 0; i < NC; ++i) v[i] = c[i];
#pragma unroll
        for (int k = 0; k < NC - 1; ++k) {
#pragma unroll
          for (int i = NC - 2; i >= k; --i) v[i] = tab[base + v[i] * q + v[i + 1]];
        }
      }
      bool dense = true;
#pragma unroll
      for (int i = 0; i < NC - 1; ++i) dense = dense && ((uint32_t)i >= d || v[i] != 0);
      if (need && !done && dense) {
#pragma unroll
        for (int i = 0; i < NC; ++i) w[i] = v[i];
        done = true;
      }
    }
    if (live) {
#pragma unroll
      for (int i = 0; i < NC; ++i) out[r * NC + i] = done ? (CT)w[i] : raw[i];
    }
    if (pid) {
      // the pattern of the row as written (classify_kernel's rule)
      uint32_t mask = 0;
      int o[NC];
#pragma unroll
      for (int i = 0; i < NC; ++i) o[i] = done ? (int)w[i] : (int)raw[i];
      const uint32_t dd = o[NC - 1] ? NC - 1 : NC - 2;
#pragma unroll
      for (int i = 0; i < NC; ++i) {
        if (live && (o[i] < 0 || o[i] >= (int)q)) bad |= 1u;
        if ((uint32_t)i < dd && o[i] != 0) mask |= 1u << i;
      }
      if (live && o[NC - 1] == 0 && o[NC - 2] == 0) bad |= 2u;
      const uint32_t pat = (o[NC - 1] ? (1u << (NC - 1)) : 0u) | mask;
      if (live) pid[r] = (uint16_t)pat;
      wave_count(hist, pat, live);
    }
  }
  if (pid) {
    if (bad) atomicOr(err, bad);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < npat; i += blockDim.x)
      if (hist[i]) atomicAdd(&counts[i], hist[i]);
  }
}

// Exclusive scans over patterns (one block of 1024 threads, npat <= 2048).
__global__ __launch_bounds__(1024) void bucket_scan_kernel(const uint32_t* __restrict__ counts, uint32_t npat,
                                                           uint32_t* __restrict__ bucket_start,
                                                           uint32_t* __restrict__ tile_start,
                                                           uint32_t* __restrict__ cursor,
                                                           uint32_t* __restrict__ ntiles,
                                                           uint32_t* __restrict__ queue) {
  __shared__ uint32_t sc[2048], st[2048];
  for (uint32_t i = threadIdx.x; i < 2048; i += blockDim.x) {
    const uint32_t c = i < npat ? counts[i] : 0;
    sc[i] = c;
    st[i] = (c + kWave - 1) / kWave;
  }
  __syncthreads();
  // Hillis-Steele inclusive scans
  for (uint32_t off = 1; off < 2048; off <<= 1) {
    uint32_t a[2], b[2];
    for (int r = 0; r < 2; ++r) {
      const uint32_t i = threadIdx.x + r * 1024;
      a[r] = (i >= off) ? sc[i - off] : 0;
      b[r] = (i >= off) ? st[i - off] : 0;
    }
    __syncthreads();
    for (int r = 0; r < 2; ++r) {
      const uint32_t i = threadIdx.x + r * 1024;
      sc[i] += a[r];
      st[i] += b[r];
    }
    __syncthreads();
  }
  for (uint32_t i = threadIdx.x; i < npat; i += blockDim.x) {
    const uint32_t c = counts[i];
    bucket_start[i] = sc[i] - c;
    tile_start[i] = st[i] - (c + kWave - 1) / kWave;
    cursor[i] = 0;
  }
  if (threadIdx.x == 0) {
    *ntiles = st[2047];
    *queue = 0;
  }
}

// tiles[t] for every tile t < ntiles: binary search of the owning pattern
__global__ void tile_fill_kernel(const uint32_t* __restrict__ counts, const uint32_t* __restrict__ bucket_start,
                                 const uint32_t* __restrict__ tile_start, uint32_t npat,
                                 const uint32_t* __restrict__ ntiles, uint64_t* __restrict__ tiles) {
  const uint32_t nt = *ntiles;
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += gridDim.x * blockDim.x) {
    uint32_t lo = 0, hi = npat;  // last pattern with tile_start <= t and a nonzero count
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (tile_start[mid] <= t) lo = mid; else hi = mid;
    }
    // tile_start is non-decreasing; skip empty patterns sharing the start
    uint32_t p = lo;
    while (p > 0 && counts[p] == 0) --p;
    const uint32_t k = t - tile_start[p];
    const uint32_t start = bucket_start[p] + k * kWave;
    const uint32_t rem = counts[p] - k * kWave;
    tiles[t] = tile_pack(p, start, rem < (uint32_t)kWave ? rem : (uint32_t)kWave);
  }
}

// perm: rows grouped by pattern.  Ranks are taken in LDS first so the global
// cursor of a pattern sees one atomic per block.
constexpr int kScatterPerThread = 16;
__global__ __launch_bounds__(256) void scatter_kernel(const uint16_t* __restrict__ pid, uint64_t n, uint32_t npat,
                                                      const uint32_t* __restrict__ bucket_start,
                                                      uint32_t* __restrict__ cursor, uint32_t* __restrict__ perm) {
  extern __shared__ uint32_t sh[];
  uint32_t* cnt = sh;          // npat
  uint32_t* base = sh + npat;  // npat
  for (uint32_t i = threadIdx.x; i < npat; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  const uint64_t chunk0 = (uint64_t)blockIdx.x * blockDim.x * kScatterPerThread;
  uint32_t rank[kScatterPerThread];
  uint32_t pat[kScatterPerThread];
#pragma unroll
  for (int r = 0; r < kScatterPerThread; ++r) {
    const uint64_t i = chunk0 + (uint64_t)r * blockDim.x + threadIdx.x;
    if (i < n) {
      pat[r] = pid[i];
      rank[r] = atomicAdd(&cnt[pat[r]], 1u);
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < npat; i += blockDim.x)
    base[i] = cnt[i] ? atomicAdd(&cursor[i], cnt[i]) : 0u;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kScatterPerThread; ++r) {
    const uint64_t i = chunk0 + (uint64_t)r * blockDim.x + threadIdx.x;
    if (i < n) perm[bucket_start[pat[r]] + base[pat[r]] + rank[r]] = (uint32_t)i;
  }
}

template <int G, typename CT>
__global__ __launch_bounds__(256) void assemble_kernel(PlanDesc P, const CT* __restrict__ codes, uint64_t n,
                                                       const uint32_t* __restrict__ lv, int32_t* __restrict__ outN) {
  constexpr int NC = 2 * G + 3;
  const uint32_t* emb1 = reinterpret_cast<const uint32_t*>(reinterpret_cast<const uint8_t*>(P.image) + P.lv[0].emb_off);
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const CT* row = codes + i * NC;
    int c0 = (int)row[0], ct = (int)row[NC - 1];
    c0 = c0 < 0 ? 0 : (c0 >= (int)P.q ? (int)P.q - 1 : c0);
    ct = ct < 0 ? 0 : (ct >= (int)P.q ? (int)P.q - 1 : ct);
    uint32_t l[G];
#pragma unroll
    for (int j = 0; j < G; ++j) l[j] = lv[i * G + j];
    int32_t out[G];
    assemble<G>(P, l, (uint32_t)c0, (uint32_t)ct, emb1[c0], emb1[ct], out);
#pragma unroll
    for (int k = 0; k < G; ++k) outN[i * G + k] = out[k];
  }
}

// ----------------------------------------------------------------------------
// factorization partition lambda(f) (Sec. 1.1, eq. 1.2; Algorithm 1 takes it
// from r^0 where it can, else by factoring)
//
// The roots found by the count give the small factors: with the orbit sweep,
// level j's zero count is the number of irreducible factors of degree exactly
// j (each contributes one Frobenius orbit of primitive roots), plus the
// factor X when c_0 = 0; with the full sweep the counts r_j = sum_{d | j}
// d n_d are Moebius-inverted.  Odd degree adds the part 1 at infinity.  The
// rest R = 2g+2 - sum_{j <= g} j n_j consists of factors of degree > g, so it
// is one factor unless R = 2g+2, where f is either irreducible or the product
// of two irreducibles of degree g+1.  Stickelberger's theorem tells them
// apart: disc f is a square in F_q iff deg f minus the number of irreducible
// factors is even.  disc f = (-1)^{D(D-1)/2} Res(f, f') / lc f with f' of
// formal degree D-1; only the parity of log Res is needed, taken along the
// Euclidean remainder sequence
// (Res(A, B) = (-1)^{deg A deg B} lc(B)^{deg A - deg R} Res(B, R)) in Zech
// arithmetic over F_q with the level-1 tables of the plan.

__device__ __forceinline__ uint32_t fq_add(const uint16_t* __restrict__ ztab, uint32_t M, uint32_t a, uint32_t b) {
  if (a == M) return b;
  if (b == M) return a;
  const uint32_t d = b >= a ? b - a : b + M - a;
  const uint32_t v = ztab[d];                    // 2 Z(d), or 6M where 1 + gamma^d = 0
  if (v == 6 * M) return M;
  const uint32_t s = a + (v >> 1);
  return s >= M ? s - M : s;
}

// fq_add without branches (the table read always issues, at index 0 when an
// operand is zero), so the reads of one quotient step go out together.
__device__ __forceinline__ uint32_t fq_add_sel(const uint16_t* __restrict__ zl, uint32_t M, uint32_t a,
                                               uint32_t b) {
  const bool az = a == M, bz = b == M;
  uint32_t d = b >= a ? b - a : b + M - a;
  d = (az || bz) ? 0u : d;
  const uint32_t v = zl[d];
  uint32_t s = a + (v >> 1);
  s = s >= M ? s - M : s;
  s = v == 6 * M ? M : s;
  return az ? b : (bz ? a : s);
}

// Parity of log disc(f) over F_q (1: disc is a nonsquare), f given by its
// codes (leading zero codes allowed); nsf is set when f and f' share a factor
// (the remainder sequence hits zero before a constant). The Euclidean
// remainder sequence of (f, f') runs as one quotient step, one leading-zero
// strip or one swap per iteration on left-aligned coefficient arrays (entry 0
// is the leading coefficient), so every array index is a compile-time
// constant and the arrays stay in registers. The parity of Res(f, f') follows
// Res(A, B) = (-1)^(deg A deg B) lc(B)^(deg A - deg R) Res(B, R), R = A mod B;
// disc f = (-1)^(n(n-1)/2) Res(f, f') / lc(f).
template <int NC>
__device__ uint32_t disc_parity(const uint32_t (&code)[NC], const uint16_t* __restrict__ zl,
                                const uint32_t* __restrict__ emb, uint32_t M, uint32_t p, uint32_t chim1,
                                bool& nsf) {
  constexpr int D = NC - 1;
  constexpr int T = 3 * D;                                  // steps: <= deg f + deg f' + stages
  uint32_t a[NC], b[NC];                                    // logs, M = the zero element
#pragma unroll
  for (int k = 0; k < NC; ++k) a[D - k] = emb[code[k]];    // a[s]: coefficient of X^(D - s)
#pragma unroll
  for (int s = 0; s < D; ++s) {                             // f': (D - s) c_(D - s) X^(D - 1 - s)
    const uint32_t li = emb[(uint32_t)(D - s) % p];         // log of the integer D - s in F_q
    b[s] = (a[s] == M || li == M) ? M : addmod(a[s], li, M);
  }
  b[D] = M;
  int dA = D, dB = D - 1;
#pragma unroll
  for (int r = 0; r < D; ++r) {                             // strip leading zeros of f and f'
    if (a[0] == M && dA > 0) {
#pragma unroll
      for (int s = 0; s < D; ++s) a[s] = a[s + 1];
      a[D] = M;
      --dA;
    }
    if (b[0] == M && dB >= 0) {
#pragma unroll
      for (int s = 0; s < D; ++s) b[s] = b[s + 1];
      b[D] = M;
      --dB;
    }
  }
  const int top = dA;
  const uint32_t lcf = a[0];
  // f' shorter than deg f - 1 (p | deg f): Res with the formal degree
  // deg f - 1 carries lc(f)^(deg f - 1 - deg f') in front
  uint32_t par = dB >= 0 ? (lcf & (uint32_t)(top - 1 - dB) & 1u) : 0u;
  bool bad = dB < 0 || lcf == M;
  bool done = bad || dB == 0;
  int dA0 = dA;                                             // deg A at the start of the stage
#pragma unroll 1
  for (int it = 0; it < T; ++it) {
    if (done) break;
    if (dA >= dB) {                                         // A -= (lc A / lc B) X^(dA - dB) B
      const bool z = a[0] == M;                             // quotient digit 0: A unchanged
      const uint32_t fac = addmod(submod(z ? 0u : a[0], b[0], M), M / 2, M);   // log of -(lc A / lc B)
#pragma unroll
      for (int s = 1; s < NC; ++s)
        a[s] = fq_add_sel(zl, M, a[s], (z || b[s] == M) ? M : addmod(fac, b[s], M));
#pragma unroll
      for (int s = 0; s < D; ++s) a[s] = a[s + 1];
      a[D] = M;
      --dA;
    } else if (dA >= 0 && a[0] == M) {                      // a leading zero of the remainder
#pragma unroll
      for (int s = 0; s < D; ++s) a[s] = a[s + 1];
      a[D] = M;
      --dA;
    } else if (dA < 0) {                                    // zero remainder: common factor
      bad = true;
      done = true;
    } else {                                                // (A, B) <- (B, A mod B)
      par ^= ((uint32_t)(dA0 * dB) & 1u) & chim1;
      par ^= b[0] & (uint32_t)(dA0 - dA) & 1u;
#pragma unroll
      for (int s = 0; s < NC; ++s) {
        const uint32_t t = a[s];
        a[s] = b[s];
        b[s] = t;
      }
      const int t = dA;
      dA = dB;
      dB = t;
      dA0 = dA;
      done = dB == 0;
    }
  }
  nsf = bad;
  if (!bad) par ^= b[0] & (uint32_t)dA & 1u;                // Res(A, c) = c^deg A
  return par ^ ((uint32_t)((top * (top - 1) / 2) & 1) & chim1) ^ (lcf & 1u);
}

// Rows per block pass of lambda_kernel (four per thread).
constexpr uint32_t kLamTile = 1024;

// The partition from the root counts r_j = #{x in F_(q^j) : f(x) = 0} (the
// zeros in lv), one block pass per kLamTile rows: the rows whose partition the
// counts leave open (deg f = 2g+2 with no factor of degree <= g: (2g+2) or
// (g+1, g+1)), or every row when sqf asks for the square-free test, are listed
// in LDS and then take the discriminant on full waves (Stickelberger: the two
// shapes differ in the character of disc f).
template <int G, typename CT>
__global__ __launch_bounds__(256) void lambda_kernel(const PlanDesc* __restrict__ Pd, const CT* __restrict__ codes,
                                                     uint64_t n, const uint32_t* __restrict__ lv,
                                                     uint32_t* __restrict__ lam, uint32_t sqf) {
  constexpr int NC = 2 * G + 3, D2 = 2 * G + 2;
  constexpr uint32_t kOpen = 1u << 30, kBad = 1u << 31;     // flags beside the partial code
  extern __shared__ uint16_t zl[];                           // the Zech table of F_q
  __shared__ uint32_t lrow[kLamTile], lpre[kLamTile];
  __shared__ uint32_t lcnt;
  const PlanDesc& P = *Pd;
  const uint32_t q = P.q, p = P.p, M = P.lv[0].M;           // level 1 is F_q
  const uint8_t* img = reinterpret_cast<const uint8_t*>(P.image);
  const uint16_t* ztab = reinterpret_cast<const uint16_t*>(img + P.lv[0].tab_off);
  const uint32_t* emb = reinterpret_cast<const uint32_t*>(img + P.lv[0].emb_off);
  const uint32_t chim1 = (M / 2) & 1u;                      // parity of log(-1)
  const bool orbit = P.orbit != 0;
  for (uint32_t k = threadIdx.x; k < M; k += blockDim.x) zl[k] = ztab[k];
  const uint32_t lane = threadIdx.x & 63u;
  for (uint64_t base = blockIdx.x * (uint64_t)kLamTile; base < n; base += (uint64_t)gridDim.x * kLamTile) {
    if (threadIdx.x == 0) lcnt = 0;
    __syncthreads();
    for (uint32_t off = 0; off < kLamTile; off += blockDim.x) {
      const uint64_t i = base + off + threadIdx.x;
      bool later = false;
      uint32_t pre = 0;
      if (i < n) {
        const CT* row = codes + i * NC;
        uint32_t code[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          int v = (int)row[k];
          code[k] = (uint32_t)(v < 0 ? 0 : (v >= (int)q ? (int)q - 1 : v));
        }
        const uint32_t x0 = code[0] == 0 ? 1u : 0u;               // X divides f
        const bool top = code[NC - 1] != 0;
        uint32_t r[G + 1], nj[G + 1];
#pragma unroll
        for (int j = 1; j <= G; ++j) r[j] = (lv[i * G + j - 1] & 0xFFu) + (orbit ? 0u : x0);
        bool ok = true;
#pragma unroll
        for (int j = 1; j <= G; ++j) {
          if (orbit) {
            nj[j] = r[j] + (j == 1 ? x0 : 0u);
          } else {
            // j n_j = sum_{d | j} mu(j / d) r_d
            int s = 0;
#pragma unroll
            for (int d = 1; d <= j; ++d) {
              if (j % d) continue;
              const int m = j / d;
              const int mu = m == 1 ? 1 : (m == 2 || m == 3) ? -1 : 0;   // j <= 4
              s += mu * (int)r[d];
            }
            ok &= s >= 0 && s % j == 0;
            nj[j] = s >= 0 ? (uint32_t)(s / j) : 0u;
          }
        }
        uint32_t c = 0, deg = 0;
        const uint32_t m1 = nj[1] + (top ? 0u : 1u);             // the part at infinity of odd degree
        c |= m1;
        deg += m1;
#pragma unroll
        for (int j = 2; j <= G; ++j) {
          c |= nj[j] << lam_shift(j);
          deg += (uint32_t)j * nj[j];
        }
        ok &= deg <= (uint32_t)D2;
        const uint32_t R = ok ? (uint32_t)D2 - deg : 0u;
        if (R > 0 && R < (uint32_t)D2) {
          ok &= R > (uint32_t)G;
          c |= 1u << lam_shift(R);
        }
        later = sqf || R == (uint32_t)D2;
        pre = c | (R == (uint32_t)D2 ? kOpen : 0u) | (ok ? 0u : kBad);
        if (!later) lam[i] = ok ? c : kLamInvalid;
      }
      const uint64_t mask = __ballot(later);                 // one LDS atomic per wave
      if (mask) {
        const uint32_t lead = (uint32_t)__builtin_ctzll(mask);
        uint32_t slot = 0;
        if (lane == lead) slot = atomicAdd(&lcnt, (uint32_t)__popcll(mask));
        slot = (uint32_t)__shfl((int)slot, (int)lead) + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
        if (later) {
          lrow[slot] = (uint32_t)(i - base);
          lpre[slot] = pre;
        }
      }
    }
    __syncthreads();
    const uint32_t nl = lcnt;
    for (uint32_t k = threadIdx.x; k < nl; k += blockDim.x) {
      const uint64_t i = base + lrow[k];
      const uint32_t pr = lpre[k];
      const CT* row = codes + i * NC;
      uint32_t code[NC];
#pragma unroll
      for (int t = 0; t < NC; ++t) {
        int v = (int)row[t];
        code[t] = (uint32_t)(v < 0 ? 0 : (v >= (int)q ? (int)q - 1 : v));
      }
      bool nsf = false;                                      // common factor with f'
      const uint32_t pd = disc_parity<NC>(code, zl, emb, M, p, chim1, nsf);
      bool ok = !(pr & kBad);
      uint32_t c = pr & ~(kOpen | kBad);
      if (pr & kOpen) {
        ok &= !nsf;
        c |= pd ? (1u << lam_shift(D2)) : (2u << lam_shift(G + 1));
      }
      lam[i] = (sqf && nsf) ? 0u : (ok ? c : kLamInvalid);  // sqf: 0 marks a row with a square factor
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// reduced representatives of Algorithm 1 (Sec. 1.2-1.3): one class is every
// row with c_d in F_q^x (codes 1..q-1), c_i = 1 (the twist-reduced choice),
// c_j one of the ncj codes in cj (when j >= 0), every position below j free,
// all other positions zero.  Row r of the class is the mixed-radix number
// (c_0, .., c_{j-1}, index of c_j, c_d - 1), c_0 least significant.

template <typename CT>
__global__ __launch_bounds__(256) void gen_reps_kernel(uint32_t q, uint32_t ncoef, uint32_t d, uint32_t i, int32_t j,
                                                       const uint32_t* __restrict__ cj, uint32_t ncj, uint64_t start,
                                                       uint64_t count, CT* __restrict__ out) {
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < count; t += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t r = start + t;
    CT* row = out + t * ncoef;
    for (uint32_t k = 0; k < ncoef; ++k) row[k] = 0;
    for (int32_t k = 0; k < j; ++k) {
      row[k] = (CT)(r % q);
      r /= q;
    }
    if (j >= 0) {
      row[j] = (CT)cj[r % ncj];
      r /= ncj;
    }
    row[i] = 1;
    row[d] = (CT)(1 + r);
  }
}

// ----------------------------------------------------------------------------
// one curve over a large field (the single-curve experiment of Table 1): the
// paper's lane-per-x layout.  Every lane takes its own x (an orbit
// representative or any nonzero element, by log), evaluates f(x) by Horner
// in absolute logs with zero-safe Zech additions (table of one period, M u32
// entries, in device memory: at F_{3001^2} it is 36 MB and lives in L2/MALL),
// and counts roots and nonsquares; waves sum by ballots, one atomic per wave.

__device__ __forceinline__ uint32_t mod_once(uint32_t v, uint32_t M) { return v >= M ? v - M : v; }

__global__ __launch_bounds__(256) void single_kernel(const uint32_t* __restrict__ zech, const uint32_t* __restrict__ xs,
                                                     uint64_t nx, SingleDesc f, unsigned long long* __restrict__ out) {
  const uint32_t M = f.M;
  uint64_t zeros = 0, odd = 0;
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < nx; t += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t x = xs ? xs[t] : (uint32_t)t;
    uint32_t acc = f.lc[f.d];
    for (int i = (int)f.d - 1; i >= 0; --i) {
      acc = acc == M ? M : mod_once(acc + x, M);          // times x
      const uint32_t c = f.lc[i];
      if (c == M) continue;                               // zero coefficient
      if (acc == M) { acc = c; continue; }
      // acc + c = c (1 + gamma^(acc - c))
      const uint32_t z = zech[acc >= c ? acc - c : acc + M - c];
      acc = z == M ? M : mod_once(c + z, M);
    }
    zeros += acc == M;
    odd += (acc != M) & (acc & 1u);
  }
  // wave sums, then one atomic per wave
  for (int off = 32; off > 0; off >>= 1) {
    zeros += __shfl_down(zeros, off);
    odd += __shfl_down(odd, off);
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    atomicAdd(out, (unsigned long long)zeros);
    atomicAdd(out + 1, (unsigned long long)odd);
  }
}

// ----------------------------------------------------------------------------
// host-callable launchers (C++ linkage, used by capi.cpp)

// The count and batch kernels of each genus are built in their own
// translation unit (count_g1.hip .. count_g4.hip, see count_entry.h).
hipError_t prepare_kernels() {
  hipError_t e = CountEntry<1>::prepare();
  if (e == hipSuccess) e = CountEntry<2>::prepare();
  if (e == hipSuccess) e = CountEntry<3>::prepare();
  if (e == hipSuccess) e = CountEntry<4>::prepare();
  return e;
}

hipError_t launch_count(const PlanDesc& P, const PlanDesc* dP, int coeff_bytes, const void* codes, const uint32_t* perm,
                        const uint64_t* tiles, const uint32_t* ntiles, uint32_t* queue, uint32_t lo, uint32_t hi,
                        int32_t* outN, uint32_t* outLv, uint32_t plog, uint32_t* acc, uint32_t* done, uint32_t grid,
                        uint32_t block, uint32_t wpe, hipStream_t s) {
#define HWC_CASE(GG)                                                                                         \
  case GG:                                                                                                   \
    return CountEntry<GG>::launch(P, dP, coeff_bytes, codes, perm, tiles, ntiles, queue, lo, hi, outN, outLv, \
                                  plog, acc, done, grid, block, wpe, s);
  switch (P.g) {
    HWC_CASE(1) HWC_CASE(2) HWC_CASE(3) HWC_CASE(4)
    default: return hipErrorInvalidValue;
  }
#undef HWC_CASE
}

hipError_t launch_batch(const JobDesc* jobs, uint32_t njobs, uint32_t gmax, uint32_t lds_bytes, uint32_t grid,
                        uint32_t block, hipStream_t s) {
  const uint32_t slot = (lds_bytes + 15u) & ~15u;
  switch (gmax) {
    case 1: return CountEntry<1>::batch(jobs, njobs, slot, grid, block, s);
    case 2: return CountEntry<2>::batch(jobs, njobs, slot, grid, block, s);
    case 3: return CountEntry<3>::batch(jobs, njobs, slot, grid, block, s);
    case 4: return CountEntry<4>::batch(jobs, njobs, slot, grid, block, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t occupancy_batch(uint32_t gmax, uint32_t block, uint32_t lds_bytes, int* blocks_per_cu) {
  const size_t lds = ((lds_bytes + 15u) & ~15u) + 16;
  switch (gmax) {
    case 1: return CountEntry<1>::occupancy_batch(block, lds, blocks_per_cu);
    case 2: return CountEntry<2>::occupancy_batch(block, lds, blocks_per_cu);
    case 3: return CountEntry<3>::occupancy_batch(block, lds, blocks_per_cu);
    case 4: return CountEntry<4>::occupancy_batch(block, lds, blocks_per_cu);
    default: return hipErrorInvalidValue;
  }
}

hipError_t occupancy_count(uint32_t g, int coeff_bytes, uint32_t block, uint32_t lds_bytes, uint32_t wpe,
                           int* blocks_per_cu) {
  switch (g) {
    case 1: return CountEntry<1>::occupancy(coeff_bytes, block, lds_bytes, wpe, blocks_per_cu);
    case 2: return CountEntry<2>::occupancy(coeff_bytes, block, lds_bytes, wpe, blocks_per_cu);
    case 3: return CountEntry<3>::occupancy(coeff_bytes, block, lds_bytes, wpe, blocks_per_cu);
    case 4: return CountEntry<4>::occupancy(coeff_bytes, block, lds_bytes, wpe, blocks_per_cu);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_assemble(const PlanDesc& P, int coeff_bytes, const void* codes, uint64_t n, const uint32_t* lv,
                           int32_t* outN, hipStream_t s) {
  const uint32_t grid = (uint32_t)((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
  if (grid == 0) return hipSuccess;
#define HWC_ASM(GG)                                                                                             \
  case GG:                                                                                                      \
    if (coeff_bytes == 1)                                                                                       \
      hipLaunchKernelGGL((assemble_kernel<GG, int8_t>), dim3(grid), dim3(256), 0, s, P,                         \
                         static_cast<const int8_t*>(codes), n, lv, outN);                                       \
    else                                                                                                        \
      hipLaunchKernelGGL((assemble_kernel<GG, int16_t>), dim3(grid), dim3(256), 0, s, P,                        \
                         static_cast<const int16_t*>(codes), n, lv, outN);                                      \
    break;
  switch (P.g) {
    HWC_ASM(1) HWC_ASM(2) HWC_ASM(3) HWC_ASM(4)
    default: return hipErrorInvalidValue;
  }
#undef HWC_ASM
  return hipGetLastError();
}

hipError_t launch_fill(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint32_t grid = (uint32_t)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

// pid (may be null): also classify the rows written into pid, counts (rows
// per pattern, added to; the caller clears it) and err, as classify_kernel
hipError_t launch_shift(int coeff_bytes, uint32_t g, const void* in, uint64_t n, uint32_t q, const uint32_t* step,
                        void* out, uint16_t* pid, uint32_t* counts, uint32_t* err, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (q > kShiftMaxQ || q < 3) return hipErrorInvalidValue;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((n + 255) / 256, 4096);
  bool prime = true;
  for (uint32_t d = 2; d * d <= q; ++d) prime = prime && q % d != 0;
  const uint32_t qm = ((1u << 20) + q - 1) / q;
  const uint32_t lds = (prime ? 0u : (q * q * q + 15) / 16 * 16) + (pid ? 4u * pattern_count(g) : 0u);
#define HWC_SHIFT1(GG, CT, DOT)                                                                          \
  hipLaunchKernelGGL((shift_kernel<2 * GG + 3, CT, DOT>), dim3(grid), dim3(256), lds, s,                  \
                     static_cast<const CT*>(in), n, q, step, static_cast<CT*>(out), pid, counts, err, qm)
#define HWC_SHIFT(GG)                                                                                       \
  case GG:                                                                                                  \
    if (coeff_bytes == 1) {                                                                                 \
      if (prime) HWC_SHIFT1(GG, int8_t, true);                                                              \
      else HWC_SHIFT1(GG, int8_t, false);                                                                   \
    } else {                                                                                                \
      if (prime) HWC_SHIFT1(GG, int16_t, true);                                                             \
      else HWC_SHIFT1(GG, int16_t, false);                                                                  \
    }                                                                                                       \
    break;
  switch (g) {
    HWC_SHIFT(1) HWC_SHIFT(2) HWC_SHIFT(3) HWC_SHIFT(4)
    default: return hipErrorInvalidValue;
  }
#undef HWC_SHIFT
#undef HWC_SHIFT1
  return hipGetLastError();
}

// classified: pid and counts were written by launch_shift (counts cleared
// before it), so the classification pass is skipped
hipError_t launch_bucket(int coeff_bytes, const void* codes, uint64_t n, uint32_t q, uint32_t g, uint16_t* pid,
                         uint32_t* counts, uint32_t* err, uint32_t* bucket_start, uint32_t* tile_start,
                         uint32_t* cursor, uint32_t* ntiles, uint32_t* queue, uint64_t* tiles, uint32_t* perm,
                         uint64_t max_tiles, bool classified, hipStream_t s) {
  const uint32_t npat = pattern_count(g);
  hipError_t e = hipSuccess;
  if (!classified) e = launch_fill(counts, 0, npat, s);
  if (e != hipSuccess) return e;
  if (n > 0 && !classified) {
    const uint32_t grid = (uint32_t)((n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048);
    if (coeff_bytes == 1)
      hipLaunchKernelGGL(classify_kernel<int8_t>, dim3(grid), dim3(256), npat * 4, s,
                         static_cast<const int8_t*>(codes), n, q, g, pid, counts, err);
    else
      hipLaunchKernelGGL(classify_kernel<int16_t>, dim3(grid), dim3(256), npat * 4, s,
                         static_cast<const int16_t*>(codes), n, q, g, pid, counts, err);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(bucket_scan_kernel, dim3(1), dim3(1024), 0, s, counts, npat, bucket_start, tile_start, cursor,
                     ntiles, queue);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (n == 0) return hipSuccess;
  {
    const uint32_t grid = (uint32_t)((max_tiles + 255) / 256 < 4096 ? (max_tiles + 255) / 256 : 4096);
    hipLaunchKernelGGL(tile_fill_kernel, dim3(grid), dim3(256), 0, s, counts, bucket_start, tile_start, npat, ntiles,
                       tiles);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  {
    const uint64_t per_block = 256ull * kScatterPerThread;
    const uint32_t grid = (uint32_t)((n + per_block - 1) / per_block);
    hipLaunchKernelGGL(scatter_kernel, dim3(grid), dim3(256), 2 * npat * 4, s, pid, n, npat, bucket_start, cursor,
                       perm);
    e = hipGetLastError();
  }
  return e;
}


hipError_t launch_lambda(const PlanDesc& P, const PlanDesc* dP, int coeff_bytes, const void* codes, uint64_t n,
                         const uint32_t* lv, uint32_t* lam, uint32_t sqf, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((n + kLamTile - 1) / kLamTile, 65536);
  const size_t lds = ((size_t)P.lv[0].M * 2 + 3) & ~size_t(3);
#define HWC_LAM(GG)                                                                                        \
  case GG:                                                                                                 \
    if (coeff_bytes == 1)                                                                                  \
      hipLaunchKernelGGL((lambda_kernel<GG, int8_t>), dim3(grid), dim3(256), lds, s, dP,                    \
                         static_cast<const int8_t*>(codes), n, lv, lam, sqf);                             \
    else                                                                                                   \
      hipLaunchKernelGGL((lambda_kernel<GG, int16_t>), dim3(grid), dim3(256), lds, s, dP,                   \
                         static_cast<const int16_t*>(codes), n, lv, lam, sqf);                            \
    break;
  switch (P.g) {
    HWC_LAM(1) HWC_LAM(2) HWC_LAM(3) HWC_LAM(4)
    default: return hipErrorInvalidValue;
  }
#undef HWC_LAM
  return hipGetLastError();
}


hipError_t launch_gen_reps(int coeff_bytes, uint32_t q, uint32_t ncoef, uint32_t d, uint32_t i, int32_t j,
                           const uint32_t* cj, uint32_t ncj, uint64_t start, uint64_t count, void* out,
                           hipStream_t s) {
  if (count == 0) return hipSuccess;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((count + 255) / 256, 65536);
  if (coeff_bytes == 1)
    hipLaunchKernelGGL(gen_reps_kernel<int8_t>, dim3(grid), dim3(256), 0, s, q, ncoef, d, i, j, cj, ncj, start,
                       count, static_cast<int8_t*>(out));
  else
    hipLaunchKernelGGL(gen_reps_kernel<int16_t>, dim3(grid), dim3(256), 0, s, q, ncoef, d, i, j, cj, ncj, start,
                       count, static_cast<int16_t*>(out));
  return hipGetLastError();
}


hipError_t launch_single(const uint32_t* zech, const uint32_t* xs, uint64_t nx, const SingleDesc& f,
                         unsigned long long* out, hipStream_t s) {
  if (nx == 0) return hipSuccess;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((nx + 255) / 256, 256 * 64);
  hipLaunchKernelGGL(single_kernel, dim3(grid), dim3(256), 0, s, zech, xs, nx, f, out);
  return hipGetLastError();
}

}  // namespace hwc
