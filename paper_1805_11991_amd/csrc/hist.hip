// Histogram of point-count tuples (the multiplicities of eq. 1.2, without the
// factorization partition): every curve's (N_1..N_g) becomes one integer key
// in mixed radix with N_1 most significant, keys are sorted by a stable LSD
// radix sort, equal runs are merged, and the keys are decoded back into
// tuples.  The result is in lexicographic order of the tuples.
//
// Radix R_k = 2 q^k + 3 covers every possible N_k (at most two affine points
// per x and two at infinity), so the key needs no Weil bound and stays valid
// for any input row.  With the partition as last column, its digit is the
// code's rank among the partition codes of 2g+2 (a few dozen values), so the
// key keeps to 32 bits where the counts leave room.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.h"

namespace hwc {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;  // keys per block
constexpr int kScanTile = 4096;

struct KeyRadix {
  uint32_t g;          // columns taken from N
  uint32_t width;      // g, or g + 1 with the factorization code as last column
  uint64_t radix[5];   // R_k, then the number of partition codes
  uint32_t nlam;       // partition codes (ascending): the code's digit is its rank
  uint32_t lam_codes[kLamCodesMax];
  uint32_t lam_mul;    // slot (c * lam_mul) >> 24 is distinct for every code c
  uint8_t lam_slot[256];   // rank + 1 of the code in that slot, 0 for none
};

// ---- device-wide exclusive scan of u32 (chunks of kScanTile) ----

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  // sh: blockDim.x entries
  const uint32_t t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (uint32_t off = 1; off < blockDim.x; off <<= 1) {
    const uint32_t a = t >= off ? sh[t - off] : 0u;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  const uint32_t incl = sh[t];
  *total = sh[blockDim.x - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(256) void scan_reduce_kernel(const uint32_t* __restrict__ in, uint64_t n,
                                                          uint32_t* __restrict__ sums) {
  __shared__ uint32_t sh[256];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  uint32_t s = 0;
  for (uint32_t j = threadIdx.x; j < (uint32_t)kScanTile; j += blockDim.x) {
    const uint64_t i = base + j;
    if (i < n) s += in[i];
  }
  uint32_t tot;
  block_exclusive_scan(s, sh, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// in and out may be the same array: each thread reads its own run before writing it
// Each thread owns 16 consecutive values, moved as four 16-byte vectors when
// the tile is whole (tiles start at multiples of 4096 values, so 16-byte aligned).
// A tile's offset is the sum of the tile sums before it (sums: one per tile,
// from scan_reduce_kernel; nullptr for a single tile); the last tile writes
// the grand total to *total when given.
__global__ __launch_bounds__(256) void scan_apply_kernel(const uint32_t* in, uint64_t n,
                                                         const uint32_t* __restrict__ sums, uint32_t* out,
                                                         uint32_t* __restrict__ total) {
  __shared__ uint32_t sh[256];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  uint32_t before = 0;
  if (sums) {
    uint32_t p = 0;
    for (uint32_t k = threadIdx.x; k < blockIdx.x; k += blockDim.x) p += sums[k];
    block_exclusive_scan(p, sh, &before);
  }
  constexpr uint32_t per = kScanTile / 256;
  const bool whole = base + kScanTile <= n;
  uint32_t v[per];
  uint32_t s = 0;
  const uint64_t first = base + threadIdx.x * per;
  if (whole) {
#pragma unroll
    for (uint32_t j = 0; j < per / 4; ++j) {
      const uint4 w = reinterpret_cast<const uint4*>(in + first)[j];
      v[4 * j] = w.x; v[4 * j + 1] = w.y; v[4 * j + 2] = w.z; v[4 * j + 3] = w.w;
    }
  } else {
#pragma unroll
    for (uint32_t j = 0; j < per; ++j) v[j] = first + j < n ? in[first + j] : 0u;
  }
#pragma unroll
  for (uint32_t j = 0; j < per; ++j) s += v[j];
  uint32_t tot;
  uint32_t off = block_exclusive_scan(s, sh, &tot) + before;
  if (total && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) *total = before + tot;
#pragma unroll
  for (uint32_t j = 0; j < per; ++j) {
    const uint32_t x = v[j];
    v[j] = off;
    off += x;
  }
  if (whole) {
#pragma unroll
    for (uint32_t j = 0; j < per / 4; ++j)
      reinterpret_cast<uint4*>(out + first)[j] = make_uint4(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
  } else {
#pragma unroll
    for (uint32_t j = 0; j < per; ++j)
      if (first + j < n) out[first + j] = v[j];
  }
}

// ---- stable LSD radix sort of u32 or u64 keys (u32 when the key fits) ----

// The tile of workgroup b among nb: workgroups go to the 8 XCDs in turn, so
// this gives each XCD a contiguous range of tiles, and the [digit][tile]
// entries that neighbouring tiles read and write share that XCD's L2 lines.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t nb) {
  const uint32_t x = b & 7u, per = nb >> 3, rem = nb & 7u;
  return x * per + (x < rem ? x : rem) + (b >> 3);
}

// The valid lanes of the wave whose digit equals this lane's (one ballot per
// digit bit).
template <int RB>
__device__ __forceinline__ uint64_t digit_peers(bool valid, uint32_t dig) {
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    const uint64_t ones = __ballot(((dig >> b) & 1u) != 0);
    peers &= ((dig >> b) & 1u) ? ones : ~ones;
  }
  return peers;
}

// top: the keys' most significant digit, which takes few values (N_1
// leads the key and clusters around q + 1): one LDS add per distinct digit of
// a wave instead of per-lane adds that would serialize on one counter.  The
// lower digits are spread out, and per-lane adds cost less than the ballots.
template <typename K, int RB>
__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const K* __restrict__ keys, uint64_t n,
                                                                  uint32_t shift, uint32_t nblocks,
                                                                  uint32_t* __restrict__ bh, bool top) {
  constexpr uint32_t kRadixBins = 1u << RB;
  __shared__ uint32_t cnt[kRadixBins];
  for (uint32_t i = threadIdx.x; i < kRadixBins; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  const uint32_t tile = xcd_tile(blockIdx.x, nblocks);
  const uint64_t base = (uint64_t)tile * kSortTile;
  K v[kSortItems];                                   // all loads in flight before the adds
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const uint64_t i = base + (uint64_t)r * kSortThreads + threadIdx.x;
    v[r] = i < n ? keys[i] : (K)0;
  }
  if (top) {   // uniform branch
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
      const bool valid = base + (uint64_t)r * kSortThreads + threadIdx.x < n;
      const uint32_t dig = (uint32_t)((v[r] >> shift) & (kRadixBins - 1));
      const uint64_t peers = digit_peers<RB>(valid, dig);
      if (valid && (peers & lt) == 0) atomicAdd(&cnt[dig], (uint32_t)__popcll(peers));
    }
  } else {
#pragma unroll
    for (int r = 0; r < kSortItems; ++r)
      if (base + (uint64_t)r * kSortThreads + threadIdx.x < n) atomicAdd(&cnt[(v[r] >> shift) & (kRadixBins - 1)], 1u);
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < kRadixBins; d += blockDim.x) bh[(uint64_t)d * nblocks + tile] = cnt[d];
}

// Keys of one sort tile (the tile of this workgroup, as in radix_hist_kernel),
// with the tile's counts of the first digit (bits 0..RB-1) into bh, so the
// first pass needs no histogram kernel.  K = u32 keys take u32 arithmetic
// (every partial key is at most the final one).  G = kr.g.
template <typename K, int RB, int G>
__global__ __launch_bounds__(kSortThreads) void make_keys_kernel(const int32_t* __restrict__ N,
                                                                 const uint32_t* __restrict__ lam, uint64_t n,
                                                                 KeyRadix kr, K* __restrict__ keys,
                                                                 uint32_t* __restrict__ err, uint32_t nblocks,
                                                                 uint32_t* __restrict__ bh) {
  constexpr uint32_t kRadixBins = 1u << RB;
  __shared__ uint32_t codes[kLamCodesMax];
  __shared__ uint8_t slots[256];
  __shared__ uint32_t cnt[kRadixBins];
  for (uint32_t t = threadIdx.x; t < kr.nlam; t += blockDim.x) codes[t] = kr.lam_codes[t];
  for (uint32_t t = threadIdx.x; t < 256; t += blockDim.x) slots[t] = kr.lam_slot[t];
  for (uint32_t t = threadIdx.x; t < kRadixBins; t += blockDim.x) cnt[t] = 0;
  __syncthreads();
  const uint32_t tile = xcd_tile(blockIdx.x, nblocks);
  const uint64_t base = (uint64_t)tile * kSortTile;
  uint32_t bad = 0;
  K kv[kSortItems];                                  // every row's loads before the stores and adds
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const uint64_t i = base + (uint64_t)r * kSortThreads + threadIdx.x;
    K key = 0;
    if (i < n) {
#pragma unroll
      for (int k = 0; k < G; ++k) {
        int32_t v = N[i * G + k];
        if (v < 0 || (uint64_t)v >= kr.radix[k]) { bad = 1; v = 0; }
        key = key * (K)kr.radix[k] + (K)v;
      }
      if (lam) {
        const uint32_t v = lam[i];
        uint32_t rk = slots[(v * kr.lam_mul) >> 24];  // rank + 1 of the code in v's slot
        if (rk == 0 || codes[rk - 1] != v) { bad = 1; rk = 1; }
        key = key * (K)kr.radix[kr.g] + (K)(rk - 1);
      }
    }
    kv[r] = key;
  }
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const uint64_t i = base + (uint64_t)r * kSortThreads + threadIdx.x;
    if (i < n) {
      keys[i] = kv[r];
      atomicAdd(&cnt[(uint32_t)kv[r] & (kRadixBins - 1)], 1u);
    }
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < kRadixBins; d += blockDim.x) bh[(uint64_t)d * nblocks + tile] = cnt[d];
  if (bad) atomicOr(err, 4u);
}

// Wave w of a block ranks the keys w*1024 .. w*1024+1023 of the block's tile
// in 16 rounds of 64 (index order within the wave): lanes with equal digits
// are found by bit ballots, and the wave keeps its own running count per digit
// in LDS, so the rounds need no block barrier.  The waves' counts then give
// each wave its start per digit, each key goes to its place in the block's
// digit-sorted tile in LDS, and the tile is written out in that order, so
// neighbouring threads store to neighbouring addresses of one digit's run
// instead of scattering single keys.
template <typename K, int RB>
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(const K* __restrict__ in, uint64_t n,
                                                                     uint32_t shift, uint32_t nblocks,
                                                                     const uint32_t* __restrict__ bh_scanned,
                                                                     K* __restrict__ out) {
  constexpr int kWaves = kSortThreads / 64;
  constexpr uint32_t kRadixBins = 1u << RB;
  constexpr uint32_t kNone = ~0u;
  __shared__ uint32_t gstart[kRadixBins];   // the block's first global position per digit
  __shared__ uint32_t lstart[kRadixBins];   // its first position per digit within the tile
  __shared__ uint32_t wrun[kWaves][kRadixBins];   // a wave's count per digit, then its start
  __shared__ K tile[kSortTile];
  __shared__ uint32_t scan_sh[kSortThreads];
  const uint32_t t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const uint32_t tb = xcd_tile(blockIdx.x, nblocks);
  const uint64_t base = (uint64_t)tb * kSortTile;
  const uint64_t nbh = (uint64_t)nblocks * kRadixBins;
  for (uint32_t d = t; d < (uint32_t)(kWaves * kRadixBins); d += blockDim.x) (&wrun[0][0])[d] = 0;
  // the wave's keys: loads issued first, so they overlap the offset reads and
  // the scan below
  const uint64_t wfirst = base + (uint64_t)wave * (kSortTile / kWaves);
  K key[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const uint64_t i = wfirst + (uint64_t)r * 64 + lane;
    key[r] = i < n ? in[i] : (K)0;
  }
  // digit counts of this block from the scanned histogram (differences of
  // consecutive entries of the [digit][block] order), then their prefix
  constexpr uint32_t kPer = kRadixBins / kSortThreads;
  uint32_t cnt[kPer], csum = 0;
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    const uint32_t d = t * kPer + k;
    const uint64_t idx = (uint64_t)d * nblocks + tb;
    const uint32_t a = bh_scanned[idx];
    const uint32_t b = idx + 1 < nbh ? bh_scanned[idx + 1] : (uint32_t)n;
    gstart[d] = a;
    cnt[k] = b - a;
    csum += cnt[k];
  }
  {
    scan_sh[t] = csum;
    __syncthreads();
    for (uint32_t off = 1; off < kSortThreads; off <<= 1) {
      const uint32_t a = t >= off ? scan_sh[t - off] : 0u;
      __syncthreads();
      scan_sh[t] += a;
      __syncthreads();
    }
    uint32_t acc = scan_sh[t] - csum;
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
      lstart[t * kPer + k] = acc;
      acc += cnt[k];
    }
  }
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t rank[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const uint64_t i = wfirst + (uint64_t)r * 64 + lane;
    const bool valid = i < n;
    const uint32_t dig = (uint32_t)((key[r] >> shift) & (kRadixBins - 1));
    const uint64_t peers = digit_peers<RB>(valid, dig);
    // every lane reads the wave's count before its leader adds the round's
    // keys (one wave: LDS operations complete in issue order)
    const uint32_t before = valid ? wrun[wave][dig] : 0u;
    const uint32_t below = (uint32_t)__popcll(peers & lt);
    __builtin_amdgcn_wave_barrier();
    if (valid && below == 0) wrun[wave][dig] = before + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
    rank[r] = valid ? before + below : kNone;
  }
  __syncthreads();
  for (uint32_t d = t; d < kRadixBins; d += blockDim.x) {   // wave starts per digit
    uint32_t acc = lstart[d];
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = wrun[w][d];
      wrun[w][d] = acc;
      acc += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    if (rank[r] == kNone) continue;
    const uint32_t dig = (uint32_t)((key[r] >> shift) & (kRadixBins - 1));
    tile[wrun[wave][dig] + rank[r]] = key[r];
  }
  __syncthreads();
  const uint32_t nin = (uint32_t)((n - base) < (uint64_t)kSortTile ? (n - base) : (uint64_t)kSortTile);
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const uint32_t j = (uint32_t)r * kSortThreads + t;
    if (j >= nin) break;
    const K key = tile[j];
    const uint32_t dig = (uint32_t)((key >> shift) & (kRadixBins - 1));
    out[gstart[dig] + (j - lstart[dig])] = key;
  }
}

// ---- run-length encoding of sorted keys ----
// Tiles of kRunTile keys, kRunItems consecutive keys per thread; a key is a
// run head when it is the first key or differs from its predecessor.

constexpr int kRunItems = 16;
constexpr int kRunTile = 256 * kRunItems;

// The thread's keys first .. first + kRunItems - 1 (16-byte loads when all
// are in range; first is a multiple of kRunItems, the buffer 256-aligned) and
// the key before them (0 at the start: key 0 is a head by its index).
template <typename K>
__device__ __forceinline__ K load_run(const K* __restrict__ keys, uint64_t first, uint64_t n, K (&v)[kRunItems]) {
  if (first + kRunItems <= n) {
    constexpr int kVec = kRunItems * (int)sizeof(K) / 16;
    const uint4* p = reinterpret_cast<const uint4*>(keys + first);
    uint4 w[kVec];
#pragma unroll
    for (int k = 0; k < kVec; ++k) w[k] = p[k];
    __builtin_memcpy(v, w, sizeof(v));
  } else {
#pragma unroll
    for (int j = 0; j < kRunItems; ++j) v[j] = first + j < n ? keys[first + j] : (K)0;
  }
  return (first > 0 && first <= n) ? keys[first - 1] : (K)0;
}

template <typename K>
__device__ __forceinline__ uint32_t run_heads(const K (&v)[kRunItems], K prev, uint64_t first, uint64_t n) {
  uint32_t c = 0;
#pragma unroll
  for (int j = 0; j < kRunItems; ++j) {
    const uint64_t i = first + j;
    c += (i < n && (i == 0 || v[j] != (j ? v[j - 1] : prev))) ? 1u : 0u;
  }
  return c;
}

// Run heads per tile.
template <typename K>
__global__ __launch_bounds__(256) void run_heads_kernel(const K* __restrict__ keys, uint64_t n,
                                                        uint32_t* __restrict__ tile_heads) {
  __shared__ uint32_t sh[256];
  const uint64_t first = (uint64_t)blockIdx.x * kRunTile + (uint64_t)threadIdx.x * kRunItems;
  K v[kRunItems];
  const K prev = load_run(keys, first, n, v);
  uint32_t tot;
  block_exclusive_scan(run_heads(v, prev, first, n), sh, &tot);
  if (threadIdx.x == 0) tile_heads[blockIdx.x] = tot;
}

// Each run head i gets its run index j (the tile's offset plus the heads
// before it in the tile): starts[j] = i, and the key decoded into the tuple
// when j < cap; counts are finished by runs_count_kernel.
template <typename K>
__global__ __launch_bounds__(256) void runs_kernel(const K* __restrict__ keys, uint64_t n,
                                                   const uint32_t* __restrict__ tile_off, KeyRadix kr, uint64_t cap,
                                                   int32_t* __restrict__ out_keys, uint64_t* __restrict__ starts) {
  __shared__ uint32_t sh[256];
  const uint64_t first = (uint64_t)blockIdx.x * kRunTile + (uint64_t)threadIdx.x * kRunItems;
  K v[kRunItems];
  const K prev = load_run(keys, first, n, v);
  uint32_t tot;
  uint64_t j = (uint64_t)tile_off[blockIdx.x] + block_exclusive_scan(run_heads(v, prev, first, n), sh, &tot);
#pragma unroll
  for (int t = 0; t < kRunItems; ++t) {
    const uint64_t i = first + t;
    if (i >= n || (i > 0 && v[t] == (t ? v[t - 1] : prev))) continue;
    starts[j] = i;
    if (j < cap) {
      K key = v[t];                                  // u32 keys: 32-bit divisions (every radix fits)
      for (int k = (int)kr.width - 1; k >= 0; --k) {
        const K r = (K)kr.radix[k];
        const uint32_t d = (uint32_t)(key % r);
        out_keys[j * kr.width + k] = (int32_t)(k == (int)kr.g ? kr.lam_codes[d] : d);
        key /= r;
      }
    }
    ++j;
  }
}

__global__ __launch_bounds__(256) void runs_count_kernel(const uint64_t* __restrict__ starts,
                                                         const uint32_t* __restrict__ nruns_p, uint64_t n,
                                                         uint64_t cap, uint64_t* __restrict__ out_counts,
                                                         uint64_t* __restrict__ out_len) {
  const uint64_t D = *nruns_p;
  for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < D && j < cap;
       j += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t end = (j + 1 < D) ? starts[j + 1] : n;
    out_counts[j] = end - starts[j];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && out_len) *out_len = D;
}

__global__ void hist_empty_kernel(uint64_t* out_len) {
  if (threadIdx.x == 0) *out_len = 0;
}

// ----------------------------------------------------------------------------

static uint32_t grid_for(uint64_t n, uint32_t block, uint32_t cap) {
  const uint64_t b = (n + block - 1) / block;
  return (uint32_t)(b < cap ? (b ? b : 1) : cap);
}

// bytes of scratch needed by hist_run for n keys
uint64_t hist_scratch_bytes(uint64_t n) {
  const uint64_t nb_sort = (n + kSortTile - 1) / kSortTile;
  const uint64_t nbh = nb_sort * 512;   // digits of up to 9 bits
  const uint64_t big = (n > nbh ? n : nbh);
  const uint64_t nsums = (big + kScanTile - 1) / kScanTile + 1;
  const uint64_t nt = (n + kRunTile - 1) / kRunTile;
  return 2 * n * 8                 // keys ping-pong
         + nbh * 4                 // block histograms
         + 2 * nt * 4              // run heads and offsets per run-length tile
         + n * 8                   // run starts
         + nsums * 4 + 64          // scan block sums, totals
         + 8 * 256;                // every part starts 256-byte aligned
}

static hipError_t scan_exclusive(const uint32_t* in, uint64_t n, uint32_t* out, uint32_t* sums, uint32_t* total,
                                 hipStream_t s) {
  const uint32_t nb = (uint32_t)((n + kScanTile - 1) / kScanTile);
  if (nb == 0) return hipSuccess;
  if (nb > 1) hipLaunchKernelGGL(scan_reduce_kernel, dim3(nb), dim3(256), 0, s, in, n, sums);
  hipLaunchKernelGGL(scan_apply_kernel, dim3(nb), dim3(256), 0, s, in, n, nb > 1 ? sums : nullptr, out, total);
  return hipGetLastError();
}

// The sort, run-length and decode steps of hist_run on keys of type K.
template <typename K, int RB>
static hipError_t sort_and_count(const int32_t* N, const uint32_t* lam, uint64_t n, const KeyRadix& kr,
                                 uint32_t npass, uint64_t nb_sort, uint64_t nbh, K* keysA, K* keysB,
                                 uint64_t* starts, uint32_t* bh, uint32_t* tile_heads, uint32_t* tile_off, uint32_t* sums,
                                 uint32_t* totals, int32_t* out_keys, uint64_t* out_counts, uint64_t cap,
                                 uint64_t* out_len, uint32_t* err, hipStream_t s) {
  switch (kr.g) {
#define HWC_KEYS(GG)                                                                                      \
  case GG:                                                                                                \
    hipLaunchKernelGGL((make_keys_kernel<K, RB, GG>), dim3((uint32_t)nb_sort), dim3(kSortThreads), 0, s, N, lam, n, \
                       kr, keysA, err, (uint32_t)nb_sort, bh);                                           \
    break;
    HWC_KEYS(1) HWC_KEYS(2) HWC_KEYS(3) HWC_KEYS(4)
#undef HWC_KEYS
    default: return hipErrorInvalidValue;
  }
  for (uint32_t pass = 0; pass < npass; ++pass) {
    const uint32_t shift = pass * RB;
    if (pass > 0)   // the first digit's counts come from make_keys_kernel
      hipLaunchKernelGGL((radix_hist_kernel<K, RB>), dim3((uint32_t)nb_sort), dim3(kSortThreads), 0, s, keysA, n,
                         shift, (uint32_t)nb_sort, bh, pass + 1 == npass);
    hipError_t e = scan_exclusive(bh, nbh, bh, sums, nullptr, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((radix_scatter_kernel<K, RB>), dim3((uint32_t)nb_sort), dim3(kSortThreads), 0, s, keysA, n, shift,
                       (uint32_t)nb_sort, bh, keysB);
    K* tmp = keysA; keysA = keysB; keysB = tmp;
  }
  const uint32_t nt = (uint32_t)((n + kRunTile - 1) / kRunTile);
  hipLaunchKernelGGL(run_heads_kernel<K>, dim3(nt), dim3(256), 0, s, keysA, n, tile_heads);
  hipError_t e = scan_exclusive(tile_heads, nt, tile_off, sums, totals, s);   // tile offsets, total runs
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(runs_kernel<K>, dim3(nt), dim3(256), 0, s, keysA, n, tile_off, kr, cap, out_keys, starts);
  hipLaunchKernelGGL(runs_count_kernel, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, starts, totals, n, cap,
                     out_counts, out_len);
  return hipGetLastError();
}

// Histogram of N[n][g] (and, when lam is given, the factorization codes
// lam[n] as a last column) into out_keys[cap][width] / out_counts[cap];
// *out_len gets the number of distinct tuples (which may exceed cap: then only
// the first cap are written).  scratch: hist_scratch_bytes(n) bytes.  err |= 4
// when a value lies outside its radix (or a code is no partition of 2g+2).
hipError_t hist_run(const int32_t* N, const uint32_t* lam, uint64_t n, uint32_t g, uint32_t q, void* scratch,
                    int32_t* out_keys, uint64_t* out_counts, uint64_t cap, uint64_t* out_len, uint32_t* err,
                    hipStream_t s) {
  if (g < 1 || g > 4) return hipErrorInvalidValue;
  KeyRadix kr;
  kr.g = g;
  kr.width = g + (lam ? 1u : 0u);
  double bits = 0;
  uint64_t qk = 1;
  for (uint32_t k = 0; k < 5; ++k) {
    if (k < 4) qk *= q;
    kr.radix[k] = (k < g) ? 2 * qk + 3 : 1;
    if (k < g) bits += __builtin_log2((double)kr.radix[k]);
  }
  kr.nlam = lam ? lam_code_list(g, kr.lam_codes) : 0u;
  kr.lam_mul = 0;
  for (uint32_t t = 0; t < 256; ++t) kr.lam_slot[t] = 0;
  if (lam) {   // an odd multiplier that puts the codes in distinct slots (the first one tried does for g <= 4)
    for (uint32_t m = 0x9E3779B1u, tries = 0; kr.lam_mul == 0; m += 2) {
      if (++tries > (1u << 16)) return hipErrorInvalidValue;
      bool clash = false;
      for (uint32_t t = 0; t < 256; ++t) kr.lam_slot[t] = 0;
      for (uint32_t r = 0; r < kr.nlam && !clash; ++r) {
        uint8_t& sl = kr.lam_slot[(kr.lam_codes[r] * m) >> 24];
        clash = sl != 0;
        sl = (uint8_t)(r + 1);
      }
      if (!clash) {
        kr.lam_mul = m;
        break;
      }
    }
  }
  if (lam) {
    kr.radix[g] = kr.nlam;
    bits += __builtin_log2((double)kr.nlam);
  }
  if (bits > 63.0) return hipErrorInvalidValue;
  const uint32_t nbits = (uint32_t)bits + 1;
  // 9-bit digits when they save a pass over 8-bit ones
  const uint32_t p8 = (nbits + 7) / 8, p9 = (nbits + 8) / 9;
  const int rb = p9 < p8 ? 9 : 8;
  const uint32_t npass = rb == 9 ? p9 : p8;
  uint8_t* p = static_cast<uint8_t*>(scratch);
  const uint64_t nb_sort = (n + kSortTile - 1) / kSortTile;
  const uint64_t nbh = nb_sort * (1u << rb);
  const uint64_t big = (n > nbh ? n : nbh);
  const uint64_t nsums = (big + kScanTile - 1) / kScanTile + 1;
  auto take = [&](uint64_t bytes) {   // 256-byte aligned parts (vector loads in the scans)
    uint8_t* q = p;
    p += (bytes + 255) / 256 * 256;
    return q;
  };
  uint64_t* keysA = reinterpret_cast<uint64_t*>(take(n * 8));
  uint64_t* keysB = reinterpret_cast<uint64_t*>(take(n * 8));
  uint64_t* starts = reinterpret_cast<uint64_t*>(take(n * 8));
  uint32_t* bh = reinterpret_cast<uint32_t*>(take(nbh * 4));
  const uint64_t nt = (n + kRunTile - 1) / kRunTile;
  uint32_t* tile_heads = reinterpret_cast<uint32_t*>(take(nt * 4));
  uint32_t* tile_off = reinterpret_cast<uint32_t*>(take(nt * 4));
  uint32_t* sums = reinterpret_cast<uint32_t*>(take(nsums * 4));
  uint32_t* totals = reinterpret_cast<uint32_t*>(take(64));
  if (n == 0) {
    if (out_len) hipLaunchKernelGGL(hist_empty_kernel, dim3(1), dim3(64), 0, s, out_len);
    return hipGetLastError();
  }
  uint32_t* keysA32 = reinterpret_cast<uint32_t*>(keysA);
  uint32_t* keysB32 = reinterpret_cast<uint32_t*>(keysB);
#define HWC_SORT(KT, RBV, A, B)                                                                                \
  return sort_and_count<KT, RBV>(N, lam, n, kr, npass, nb_sort, nbh, A, B, starts, bh, tile_heads, tile_off, sums, totals, \
                                 out_keys, out_counts, cap, out_len, err, s)
  if (nbits <= 32) {
    if (rb == 9) HWC_SORT(uint32_t, 9, keysA32, keysB32);
    HWC_SORT(uint32_t, 8, keysA32, keysB32);
  }
  if (rb == 9) HWC_SORT(uint64_t, 9, keysA, keysB);
  HWC_SORT(uint64_t, 8, keysA, keysB);
#undef HWC_SORT
}

}  // namespace hwc
