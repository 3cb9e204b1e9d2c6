// Stable LSD radix sort of (key, int32 value) pairs on gfx950, used by the
// build: the sort of every core model's items by (model, key, id) behind the
// sorted hashkey arrays (Section 3.3.1, Section 5.1) and the grouping of
// k-means members by cluster (Section 3.2).
//
// Each pass orders the items stably by one 8-bit digit of the key, lowest
// digit first, so after the passes over bits [0, bits) the items are ordered
// by those bits with ties in input order.  A pass is three launches:
//   1. digit_count_kernel: one workgroup per tile of kTile items counts the
//      tile's digits in LDS and stores the 256 counts, digit-major
//      (count[digit * ntiles + tile]).
//   2. digit_scan_kernel: one workgroup per digit turns that digit's counts
//      into their exclusive prefix sum over the tiles and stores the digit's
//      total; a (digit, tile)'s first output slot is that prefix plus the
//      totals of the smaller digits.
//   3. digit_scatter_kernel: the tile's 4 waves each own a contiguous quarter
//      of it; a wave counts its digits, the workgroup forms each wave's first
//      slot per digit (the tile's slot plus the counts of the earlier waves),
//      then each wave walks its items 64 at a time in order: the lanes with
//      equal digits find each other with 8 ballots, an item's slot is its
//      wave's running count for the digit plus the number of equal lanes
//      below it, and the lowest such lane advances the running count.  Items
//      thus keep their input order within a digit.
#include <algorithm>
#include <cstdint>

#include "lider_internal.hpp"

namespace lider {

namespace {

constexpr int kSortNT = 256;                     // threads per workgroup
constexpr int kSortWaves = kSortNT / 64;
constexpr int kPerLane = 16;                     // items per lane
constexpr int kTile = kSortNT * kPerLane;        // items per workgroup tile
constexpr int kWaveItems = kTile / kSortWaves;   // contiguous items per wave

template <class K>
__device__ inline uint32_t digit_of(K key, int shift) {
  return uint32_t(key >> shift) & 255u;
}

template <class K>
__global__ __launch_bounds__(kSortNT) void digit_count_kernel(const K* __restrict__ keys,
                                                              int64_t n, int shift,
                                                              int64_t ntiles,
                                                              uint32_t* __restrict__ count) {
  __shared__ uint32_t h[256];
  const int tid = threadIdx.x;
  h[tid] = 0u;
  __syncthreads();
  const int64_t t0 = int64_t(blockIdx.x) * kTile;
  for (int u = 0; u < kPerLane; ++u) {
    const int64_t i = t0 + int64_t(u) * kSortNT + tid;
    if (i < n) atomicAdd(&h[digit_of(keys[i], shift)], 1u);
  }
  __syncthreads();
  count[int64_t(tid) * ntiles + blockIdx.x] = h[tid];
}

// Per digit (one workgroup each): the exclusive prefix sum over the tiles of
// that digit's counts, in place, and the digit's total.  Each thread sums a
// contiguous run of tiles, the run sums are scanned in LDS, then each thread
// rewrites its run.
__global__ __launch_bounds__(kSortNT) void digit_scan_kernel(uint32_t* __restrict__ count,
                                                             int64_t ntiles,
                                                             uint32_t* __restrict__ total) {
  __shared__ uint32_t part[kSortNT];
  const int tid = threadIdx.x;
  uint32_t* v = count + int64_t(blockIdx.x) * ntiles;
  const int64_t per = (ntiles + kSortNT - 1) / kSortNT;
  const int64_t a = std::min<int64_t>(ntiles, int64_t(tid) * per);
  const int64_t e = std::min<int64_t>(ntiles, a + per);
  uint32_t s = 0;
  for (int64_t i = a; i < e; ++i) s += v[i];
  part[tid] = s;
  __syncthreads();
  for (int o = 1; o < kSortNT; o <<= 1) {  // inclusive scan of the run sums
    const uint32_t x = tid >= o ? part[tid - o] : 0u;
    __syncthreads();
    part[tid] += x;
    __syncthreads();
  }
  uint32_t acc = part[tid] - s;
  if (tid == kSortNT - 1) total[blockIdx.x] = part[tid];
  for (int64_t i = a; i < e; ++i) {
    const uint32_t x = v[i];
    v[i] = acc;
    acc += x;
  }
}

template <class K>
__global__ __launch_bounds__(kSortNT) void digit_scatter_kernel(
    const K* __restrict__ kin, const int32_t* __restrict__ vin, int64_t n, int shift,
    int64_t ntiles, const uint32_t* __restrict__ first, const uint32_t* __restrict__ total,
    K* __restrict__ kout, int32_t* __restrict__ vout) {
  __shared__ uint32_t wcount[kSortWaves][256];
  __shared__ uint32_t dbase[256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t below = (uint64_t(1) << lane) - 1;
  for (int w = 0; w < kSortWaves; ++w) wcount[w][tid] = 0u;
  // first slot of each digit: exclusive prefix of the digit totals
  dbase[tid] = total[tid];
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const uint32_t x = tid >= o ? dbase[tid - o] : 0u;
    __syncthreads();
    dbase[tid] += x;
    __syncthreads();
  }
  const uint32_t mybase = dbase[tid] - total[tid];
  // the wave's items: [w0, w0 + kWaveItems), walked 64 at a time; its keys
  // stay in registers between the counting and the scattering
  const int64_t w0 = int64_t(blockIdx.x) * kTile + int64_t(wave) * kWaveItems;
  K key[kWaveItems / 64];
#pragma unroll
  for (int u = 0; u < kWaveItems / 64; ++u) {
    const int64_t i = w0 + int64_t(u) * 64 + lane;
    key[u] = i < n ? kin[i] : K(0);
    if (i < n) atomicAdd(&wcount[wave][digit_of(key[u], shift)], 1u);
  }
  __syncthreads();
  // each wave's first slot per digit: the digit's first slot, the earlier
  // tiles' and the earlier waves' counts (thread tid handles digit tid)
  {
    uint32_t base = mybase + first[int64_t(tid) * ntiles + blockIdx.x];
    for (int w = 0; w < kSortWaves; ++w) {
      const uint32_t c = wcount[w][tid];
      wcount[w][tid] = base;
      base += c;
    }
  }
  __syncthreads();
  uint32_t* run = wcount[wave];  // the wave's next slot per digit
#pragma unroll
  for (int u = 0; u < kWaveItems / 64; ++u) {
    const int64_t i = w0 + int64_t(u) * 64 + lane;
    const bool ok = i < n;
    const uint32_t dg = digit_of(key[u], shift);
    // lanes holding the same digit (valid lanes only)
    uint64_t peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t ones = __ballot(ok && ((dg >> b) & 1u));
      peers &= ((dg >> b) & 1u) ? ones : ~ones;
    }
    uint32_t slot = 0;
    if (ok) slot = run[dg] + uint32_t(__popcll(peers & below));
    __builtin_amdgcn_wave_barrier();
    __threadfence_block();
    if (ok && (peers & below) == 0) run[dg] += uint32_t(__popcll(peers));
    __builtin_amdgcn_wave_barrier();
    __threadfence_block();
    if (ok) {
      kout[slot] = key[u];
      vout[slot] = vin[i];
    }
  }
}

int key_passes(int bits) { return (std::max(1, bits) + 7) / 8; }

}  // namespace

size_t radix_sort_temp_bytes(int64_t n, int key_bytes) {
  const int64_t ntiles = (n + kTile - 1) / kTile;
  return al256(size_t(n) * size_t(key_bytes)) + al256(size_t(n) * 4) +
         al256(size_t(ntiles) * 256 * 4) + al256(256 * 4);
}

template <class K>
int radix_sort_pairs(const K* keys_in, const int32_t* vals_in, K* keys_out, int32_t* vals_out,
                     int64_t n, int bits, void* temp, size_t temp_bytes, hipStream_t st) {
  if (n < 0 || n > INT32_MAX || bits < 1 || bits > int(8 * sizeof(K)))
    return set_error(LIDER_EINVAL, "radix sort: bad size or key width");
  if (temp_bytes < radix_sort_temp_bytes(n, int(sizeof(K))))
    return set_error(LIDER_EINVAL, "radix sort: temporary buffer too small");
  if (n == 0) return LIDER_OK;
  const int64_t ntiles = (n + kTile - 1) / kTile;
  char* p = static_cast<char*>(temp);
  K* ktmp = reinterpret_cast<K*>(p);
  p += al256(size_t(n) * sizeof(K));
  int32_t* vtmp = reinterpret_cast<int32_t*>(p);
  p += al256(size_t(n) * 4);
  uint32_t* count = reinterpret_cast<uint32_t*>(p);
  p += al256(size_t(ntiles) * 256 * 4);
  uint32_t* total = reinterpret_cast<uint32_t*>(p);
  const int P = key_passes(bits);
  const K* ks = keys_in;
  const int32_t* vs = vals_in;
  for (int pass = 0; pass < P; ++pass) {
    // the last pass writes the outputs; the buffers alternate before it
    const bool to_out = (P - 1 - pass) % 2 == 0;
    K* kd = to_out ? keys_out : ktmp;
    int32_t* vd = to_out ? vals_out : vtmp;
    const int shift = 8 * pass;
    hipLaunchKernelGGL(digit_count_kernel<K>, dim3(unsigned(ntiles)), dim3(kSortNT), 0, st, ks, n,
                       shift, ntiles, count);
    hipLaunchKernelGGL(digit_scan_kernel, dim3(256), dim3(kSortNT), 0, st, count, ntiles, total);
    hipLaunchKernelGGL(digit_scatter_kernel<K>, dim3(unsigned(ntiles)), dim3(kSortNT), 0, st, ks,
                       vs, n, shift, ntiles, count, total, kd, vd);
    ks = kd;
    vs = vd;
  }
  return check_hip(hipGetLastError(), "radix sort");
}

template int radix_sort_pairs<uint32_t>(const uint32_t*, const int32_t*, uint32_t*, int32_t*,
                                        int64_t, int, void*, size_t, hipStream_t);
template int radix_sort_pairs<uint64_t>(const uint64_t*, const int32_t*, uint64_t*, int32_t*,
                                        int64_t, int, void*, size_t, hipStream_t);

}  // namespace lider
