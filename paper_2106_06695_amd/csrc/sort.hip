// Device-wide exclusive scan of uint32 arrays and a stable LSD radix sort of
// (key, value) pairs, used by the lattice build to order points spatially and
// to group (point, vertex) entries by vertex.
//
// Radix sort: 8-bit digits, one pass per digit. A pass histograms each tile
// of kTile elements per digit (digit-major layout), scans the histograms
// across the whole grid, and scatters each tile stably: inside a wavefront,
// lanes holding the same digit are found with eight ballots (one per digit
// bit), and per-wave digit counts in LDS give the offsets across the block's
// four wavefronts, so equal keys keep their input order.
#include "sgp_internal.h"

namespace sgp {
namespace {

constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;
constexpr int kSortItems = 8;
constexpr int kTile = kBlock * kSortItems;
constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ uint32_t block_sum_u32(uint32_t v) {
  __shared__ uint32_t sh[kBlock];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  const uint32_t s = sh[0];
  __syncthreads();
  return s;
}

// Inclusive block scan (Hillis-Steele in LDS); returns the inclusive value.
__device__ __forceinline__ uint32_t block_incl_scan_u32(uint32_t v, uint32_t* total) {
  __shared__ uint32_t sh[kBlock];
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    const uint32_t add = tid >= off ? sh[tid - off] : 0u;
    __syncthreads();
    sh[tid] += add;
    __syncthreads();
  }
  const uint32_t r = sh[tid];
  *total = sh[kBlock - 1];
  __syncthreads();
  return r;
}

// Pass 1: sum of each tile.
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t count,
                                                        uint32_t* __restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  uint32_t s = 0;
  for (int it = 0; it < kScanItems; ++it) {
    const int64_t e = base + (int64_t)it * kBlock + threadIdx.x;
    if (e < count) s += in[e];
  }
  s = block_sum_u32(s);
  if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

// Pass 2: exclusive scan of the tile sums in one block (loops over chunks).
__global__ __launch_bounds__(kBlock) void k_scan_sums(uint32_t* __restrict__ sums, int64_t nt,
                                                      uint32_t* __restrict__ total) {
  uint32_t carry = 0;
  for (int64_t base = 0; base < nt; base += kBlock) {
    const int64_t e = base + threadIdx.x;
    const uint32_t v = e < nt ? sums[e] : 0u;
    uint32_t chunk;
    const uint32_t incl = block_incl_scan_u32(v, &chunk);
    if (e < nt) sums[e] = carry + incl - v;
    carry += chunk;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

// Pass 3: exclusive scan inside each tile, offset by the tile's prefix.
// Thread t owns kScanItems consecutive elements so that the order is kept.
__global__ __launch_bounds__(kBlock) void k_scan_apply(const uint32_t* __restrict__ in, int64_t count,
                                                       const uint32_t* __restrict__ sums,
                                                       uint32_t* __restrict__ out) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
  for (int u = 0; u < kScanItems; ++u) {
    const int64_t e = base + u;
    v[u] = e < count ? in[e] : 0u;
    s += v[u];
  }
  uint32_t tot;
  uint32_t run = block_incl_scan_u32(s, &tot) - s + sums[blockIdx.x];
  for (int u = 0; u < kScanItems; ++u) {
    const int64_t e = base + u;
    if (e < count) out[e] = run;
    run += v[u];
  }
}

template <typename K>
__global__ __launch_bounds__(kBlock) void k_radix_hist(const K* __restrict__ keys, int64_t count,
                                                       int shift, uint32_t* __restrict__ hist,
                                                       int64_t ntiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
  for (int it = 0; it < kSortItems; ++it) {
    const int64_t e = base + (int64_t)it * kBlock + threadIdx.x;
    if (e < count) atomicAdd(&h[(uint32_t)(keys[e] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

template <typename K>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(const K* __restrict__ keys_in,
                                                          const uint32_t* __restrict__ vals_in,
                                                          int64_t count, int shift,
                                                          const uint32_t* __restrict__ offs,
                                                          int64_t ntiles, K* __restrict__ keys_out,
                                                          uint32_t* __restrict__ vals_out) {
  __shared__ uint32_t running[256];
  __shared__ uint32_t wave_cnt[kWaves][256];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  running[tid] = 0;
  for (int w = 0; w < kWaves; ++w) wave_cnt[w][tid] = 0;
  __syncthreads();
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * kTile;
  for (int it = 0; it < kSortItems; ++it) {
    const int64_t e = base + (int64_t)it * kBlock + tid;
    const bool valid = e < count;
    K key = 0;
    uint32_t val = 0;
    uint32_t digit = 0;
    if (valid) {
      key = keys_in[e];
      val = vals_in[e];
      digit = (uint32_t)(key >> shift) & 255u;
    }
    // lanes of this wave holding the same digit
    uint64_t match = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      const uint64_t bits = __ballot(valid && ((digit >> b) & 1u));
      match &= ((digit >> b) & 1u) ? bits : ~bits;
    }
    const uint32_t rank_in_wave = (uint32_t)__popcll(match & lt_mask);
    if (valid && rank_in_wave == 0) wave_cnt[wave][digit] = (uint32_t)__popcll(match);
    __syncthreads();
    if (valid) {
      uint32_t pos = running[digit] + rank_in_wave;
      for (int w = 0; w < wave; ++w) pos += wave_cnt[w][digit];
      const int64_t dst = (int64_t)offs[(int64_t)digit * ntiles + blockIdx.x] + pos;
      keys_out[dst] = key;
      vals_out[dst] = val;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < kWaves; ++w) {
      add += wave_cnt[w][tid];
      wave_cnt[w][tid] = 0;
    }
    running[tid] += add;
    __syncthreads();
  }
}

}  // namespace

int scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t count, uint32_t* total,
                       uint32_t* tmp, hipStream_t s) {
  const int64_t nt = (count + kScanTile - 1) / kScanTile;
  if (nt < 1) return SGP_OK;
  ProfScope ps(KK_SCAN, s);
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nt), dim3(kBlock), 0, s, in, count, tmp);
  SGP_LAUNCH_CHECK("k_scan_reduce");
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, s, tmp, nt, total);
  SGP_LAUNCH_CHECK("k_scan_sums");
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nt), dim3(kBlock), 0, s, in, count, tmp, out);
  SGP_LAUNCH_CHECK("k_scan_apply");
  return SGP_OK;
}

size_t scan_tmp_words(int64_t count) { return (size_t)((count + kScanTile - 1) / kScanTile) + 1; }

size_t radix_tmp_words(int64_t count) {
  const int64_t ntiles = (count + kTile - 1) / kTile;
  const int64_t h = 256 * ntiles;
  return (size_t)(2 * h) + scan_tmp_words(h);
}

template <typename K>
int radix_sort_pairs(K* keys, uint32_t* vals, K* keys_alt, uint32_t* vals_alt, int64_t count,
                     int bits, uint32_t* tmp, hipStream_t s, bool* result_in_alt) {
  *result_in_alt = false;
  if (count <= 1 || bits <= 0) return SGP_OK;
  const int64_t ntiles = (count + kTile - 1) / kTile;
  const int64_t h = 256 * ntiles;
  uint32_t* hist = tmp;
  uint32_t* offs = tmp + h;
  uint32_t* stmp = tmp + 2 * h;
  K* kin = keys;
  uint32_t* vin = vals;
  K* kout = keys_alt;
  uint32_t* vout = vals_alt;
  int rc;
  for (int shift = 0; shift < bits; shift += 8) {
    {
      ProfScope ps(KK_SORT, s);
      hipLaunchKernelGGL((k_radix_hist<K>), dim3((unsigned)ntiles), dim3(kBlock), 0, s, kin, count,
                         shift, hist, ntiles);
      SGP_LAUNCH_CHECK("k_radix_hist");
    }
    if ((rc = scan_exclusive_u32(hist, offs, h, nullptr, stmp, s))) return rc;
    {
      ProfScope ps(KK_SORT, s);
      hipLaunchKernelGGL((k_radix_scatter<K>), dim3((unsigned)ntiles), dim3(kBlock), 0, s, kin, vin,
                         count, shift, offs, ntiles, kout, vout);
      SGP_LAUNCH_CHECK("k_radix_scatter");
    }
    K* tk = kin;
    kin = kout;
    kout = tk;
    uint32_t* tv = vin;
    vin = vout;
    vout = tv;
    *result_in_alt = !*result_in_alt;
  }
  return SGP_OK;
}

template int radix_sort_pairs<uint32_t>(uint32_t*, uint32_t*, uint32_t*, uint32_t*, int64_t, int,
                                        uint32_t*, hipStream_t, bool*);
template int radix_sort_pairs<unsigned long long>(unsigned long long*, uint32_t*, unsigned long long*,
                                                  uint32_t*, int64_t, int, uint32_t*, hipStream_t,
                                                  bool*);

}  // namespace sgp
