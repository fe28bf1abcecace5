// Lattice construction (Section 3.2, Splat and Blur):
//   k_elevate         elevation, enclosing simplex and barycentric weights
//                     of every point
//   k_point_key + radix sort
//                     points sorted by their remainder-0 lattice point, then
//                     by the ranks of their first coordinates; tiles of P
//                     consecutive sorted points
//   k_tile_insert     hash every simplex vertex of a tile, insert each
//                     distinct one into a hash table once, and keep per slot
//                     its first entry in caller order and in sorted order
//   k_mark_first / k_count_first / k_scan / k_compact
//                     number the distinct vertices by first occurrence in
//                     the caller's (point, vertex) order and write their keys
//   k_neighbors       neighbours of every lattice point along the d+1
//                     lattice directions at offsets -r..r
//   internal numbering by first touch in sorted order, then per tile the
//   runs (k_tile_order / k_tile_fill) and the pieces grouped by lattice point
//
// Hash table: open addressing with linear probing over 64-bit key hashes,
// first tried at an eighth of its worst-case size (a slot is claimed by one
// 64-bit compare-and-swap, so insertion is lock-free and never waits on
// another lane). Two distinct keys with equal
// hashes would share a slot; every entry's key is compared with its hashing
// group's first key (k_tile_insert), and that first key, in every tile that
// holds the group, with its lattice point's stored key (k_tile_order). The
// host rebuilds with a new seed if any differ, so the final lattice is
// exact.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "sgp_internal.h"

namespace sgp {
namespace {

enum BuildFlag : uint32_t {
  BF_NONFINITE = 1u,
  BF_OVERFLOW = 2u,
  BF_TABLE_FULL = 4u,
  BF_COLLISION = 8u,
  BF_ORDER = 16u  // a tile's sorted order names an entry past the tile (internal error)
};

constexpr unsigned long long kEmpty = 0ull;
constexpr uint32_t kNoFirst = 0xffffffffu;
constexpr uint32_t kCanonBit = 0x80000000u;  // slot word holds a lattice index
constexpr double kKeyLimit = 1073741824.0;   // |y_i| bound that keeps keys in int32
constexpr int kItems = 8;                    // elements per thread in the scan passes
constexpr int kChunk = kBlock * kItems;
constexpr int kScanThreads = 1024;

__device__ __forceinline__ unsigned long long mix64(unsigned long long h) {
  h ^= h >> 30;
  h *= 0xbf58476d1ce4e5b9ull;
  h ^= h >> 27;
  h *= 0x94d049bb133111ebull;
  h ^= h >> 31;
  return h;
}

// Key hash: a seeded linear form sum_l a_l v_l (mod 2^64) over the stored
// coordinates with odd coefficients a_l, then a 64-bit mix (a bijection) so
// that the low bits index the table. One 64-bit multiply per coordinate.
struct HashCoef {
  unsigned long long a[kMaxD];
};

inline HashCoef hash_coef(unsigned long long seed) {
  HashCoef c;
  unsigned long long x = seed;
  for (int l = 0; l < kMaxD; ++l) {
    x += 0x9e3779b97f4a7c15ull;  // splitmix64 sequence
    unsigned long long z = x;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    c.a[l] = (z ^ (z >> 31)) | 1ull;
  }
  return c;
}

__device__ __forceinline__ unsigned long long hash_acc(unsigned long long h, unsigned long long a, int32_t v) {
  return h + a * (unsigned long long)(long long)v;
}

__device__ __forceinline__ unsigned long long hash_final(unsigned long long h) {
  h = mix64(h);
  return h == kEmpty ? 1ull : h;
}

struct SimplexArgs {
  const float* X;
  int64_t n;
  int d;
  double f[kMaxD];
  float* w;
  int32_t* pt_r0;
  uint8_t* pt_rank;
  uint32_t* flags;
  int32_t* rmin;  // per-dimension min / max of the remainder-0 point, in units of d+1
  int32_t* rmax;
};

// Linear probing stops after maxp slots (kMaxProbe with the full table,
// kMaxProbeReduced with a reduced one): a longer sequence counts as a full
// table, and a build that started with a reduced table then retries with
// the full one. Lookups use the same bound, so they find every key that
// was inserted.
constexpr unsigned long long kMaxProbe = 4096;
constexpr unsigned long long kMaxProbeReduced = 32;

// Read-only lookup. Slot of hash h (-1 if absent), once the first probe (slot s0 = h & mask,
// which holds another hash) has been read: linear probing from s0 + 1.
__device__ int64_t table_find_from(const unsigned long long* tab, unsigned long long mask,
                                   unsigned long long h, unsigned long long maxp, unsigned long long s0) {
  unsigned long long s = (s0 + 1) & mask;
  for (unsigned long long probe = 1; probe <= mask && probe < maxp; ++probe) {
    const unsigned long long cur = tab[s];
    if (cur == h) return (int64_t)s;
    if (cur == kEmpty) return -1;
    s = (s + 1) & mask;
  }
  return -1;
}

// One point per d+1 consecutive lanes: lane j owns coordinate j of the
// elevated point and, later, vertex j of its simplex. Values other lanes
// need pass through LDS between barriers. Each floating-point operation
// rounds once (no contraction), so keys and weights are reproducible.
// Blocks take groups of P points in turn; the per-dimension range of the
// remainder-0 points is gathered in LDS and merged into the global words
// once per block (one block per group would put millions of atomics on the
// same few words).
constexpr int kElevateBlocks = 4096;
__global__ __launch_bounds__(kBlock) void k_elevate(SimplexArgs a) {
  __shared__ double sh_a[kBlock];    // scaled inputs c_j, then residuals
  __shared__ double sh_q[kBlock];    // residuals / (d+1) in rank order
  __shared__ int32_t sh_i[kBlock];   // quotients
  __shared__ int32_t sh_bad[kBlock];
  __shared__ int32_t sh_min[kMaxD], sh_max[kMaxD];
  const int d = a.d, D = d + 1;
  const int P = kBlock / D;
  const int tid = threadIdx.x;
  const int p = tid / D, j = tid - p * D;
  const int base = p * D;
  if (tid < d) {
    sh_min[tid] = INT32_MAX;
    sh_max[tid] = INT32_MIN;
  }
  const int64_t groups = (a.n + P - 1) / P;
  for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
    const int64_t i = g * P + p;
    const bool live = (p < P) && (i < a.n);
    sh_bad[tid] = 0;
    double cj = 0.0;
    if (live && j >= 1) cj = (double)a.X[i * d + (j - 1)] * a.f[j - 1];
    sh_a[tid] = cj;
    __syncthreads();

    // elevation: y_j = (c_d + c_{d-1} + ... + c_{j+1}) - j c_j, and y_0 = sum of all c
    double y = 0.0;
    if (live) {
      double S = 0.0;
      for (int l = d; l > j; --l) S = S + sh_a[base + l];
      y = (j >= 1) ? S - (double)j * cj : S;
    }
    uint32_t bad = 0;
    int32_t q = 0;
    if (live) {
      if (isnan(y) || isinf(y)) bad = BF_NONFINITE;
      else if (!(fabs(y) <= kKeyLimit)) bad = BF_OVERFLOW;
      else q = (int32_t)rint(y / (double)D);  // nearest multiple of d+1 (ties to even)
    }
    sh_i[tid] = q;
    if (bad) {
      sh_bad[base] = 1;
      atomicOr(a.flags, bad);
    }
    __syncthreads();
    const bool ok = live && sh_bad[base] == 0;

    int32_t r0 = q * D;
    int dsum = 0;
    if (ok)
      for (int l = 0; l < D; ++l) dsum += sh_i[base + l];
    double del = y - (double)r0;
    sh_a[tid] = del;
    __syncthreads();

    // rank 0 = largest residual; equal residuals rank the lower index first
    int rank = 0;
    if (ok) {
      for (int l = 0; l < D; ++l) {
        const double o = sh_a[base + l];
        rank += (o > del || (o == del && l < j)) ? 1 : 0;
      }
      // make the remainder-0 point sum to zero by moving |dsum| coordinates by d+1
      if (dsum > 0) {
        if (rank >= D - dsum) { r0 -= D; rank += dsum - D; }
        else rank += dsum;
      } else if (dsum < 0) {
        if (rank < -dsum) { r0 += D; rank += dsum + D; }
        else rank += dsum;
      }
    }
    rank = min(max(rank, 0), d);
    del = y - (double)r0;
    if (ok) sh_q[base + rank] = del / (double)D;
    if (ok && j < d) {
      atomicMin(&sh_min[j], r0 / D);
      atomicMax(&sh_max[j], r0 / D);
    }
    __syncthreads();
    if (ok) {  // a rejected point fails the build
      // barycentric weight of vertex k (= this lane): gap between consecutive
      // sorted residuals; vertex 0 takes the remainder
      const int k = j;
      const double b = (k >= 1) ? sh_q[base + d - k] - sh_q[base + d + 1 - k]
                                : sh_q[base + d] + (1.0 - sh_q[base]);
      a.w[i * D + k] = (float)b;
      if (j < d) {
        a.pt_r0[i * d + j] = r0;
        a.pt_rank[i * d + j] = (uint8_t)rank;
      }
    }
  }
  __syncthreads();
  if (tid < d && sh_min[tid] <= sh_max[tid]) {
    atomicMin(&a.rmin[tid], sh_min[tid]);
    atomicMax(&a.rmax[tid], sh_max[tid]);
  }
}

__device__ __forceinline__ int block_exclusive_scan(int v, int* total) {
  __shared__ int sh[kBlock];
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    const int add = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += add;
    __syncthreads();
  }
  const int incl = sh[tid];
  *total = sh[kBlock - 1];
  __syncthreads();
  return incl - v;
}

// First occurrences as a bitmask over entries: bit e is set when entry e
// is the first of its slot (one pass over the table's slots), so counting
// and compaction read 1 bit per entry instead of gathering from the table.
__global__ __launch_bounds__(kBlock) void k_mark_first(const uint32_t* __restrict__ first, int64_t cap,
                                                       uint32_t* __restrict__ bits) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < cap; s += stride) {
    const uint32_t v = first[s];
    if (v != kNoFirst) atomicOr(&bits[v >> 5], 1u << (v & 31));
  }
}

// The first-occurrence flags of entries e0 .. e0 + 7 (e0 a multiple of 8).
__device__ __forceinline__ uint32_t first_flags(const uint32_t* bits, int64_t e0) {
  return ((const uint8_t*)bits)[e0 >> 3];
}

__global__ __launch_bounds__(kBlock) void k_count_first(const uint32_t* __restrict__ bits, int64_t L,
                                                        uint32_t* __restrict__ counts) {
  const int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)threadIdx.x * kItems;
  const int c = base < L ? __popc(first_flags(bits, base)) : 0;
  int total;
  (void)block_exclusive_scan(c, &total);
  if (threadIdx.x == 0) counts[blockIdx.x] = (uint32_t)total;
}

// Exclusive scan of the per-block counts in one block; writes the total m.
__global__ __launch_bounds__(kScanThreads) void k_scan(const uint32_t* __restrict__ counts,
                                                       uint32_t* __restrict__ offsets, int64_t nb,
                                                       uint32_t* __restrict__ total) {
  __shared__ uint32_t sh[kScanThreads];
  const int tid = threadIdx.x;
  uint32_t carry = 0;
  for (int64_t base = 0; base < nb; base += kScanThreads) {
    const uint32_t v = (base + tid < nb) ? counts[base + tid] : 0u;
    sh[tid] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
      const uint32_t add = tid >= off ? sh[tid - off] : 0u;
      __syncthreads();
      sh[tid] += add;
      __syncthreads();
    }
    if (base + tid < nb) offsets[base + tid] = carry + sh[tid] - v;
    carry += sh[kScanThreads - 1];
    __syncthreads();
  }
  if (tid == 0) *total = carry;
}

// Stored coordinate l of vertex k of point i, from its simplex descriptor.
__device__ __forceinline__ int32_t vertex_coord(const int32_t* pt_r0, const uint8_t* pt_rank,
                                                int64_t i, int d, int k, int l) {
  return pt_r0[i * d + l] + k - ((int)pt_rank[i * d + l] > d - k ? d + 1 : 0);
}

__global__ __launch_bounds__(kBlock) void k_compact(const uint32_t* __restrict__ bits,
                                                    const int32_t* __restrict__ slot,
                                                    uint32_t* __restrict__ tab_first, int64_t L,
                                                    const uint32_t* __restrict__ offsets,
                                                    const int32_t* __restrict__ pt_r0,
                                                    const uint8_t* __restrict__ pt_rank, int d,
                                                    int64_t m, int32_t* __restrict__ keys,
                                                    uint32_t* __restrict__ flags) {
  const int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)threadIdx.x * kItems;
  const uint32_t fl = base < L ? first_flags(bits, base) : 0u;
  int total;
  uint32_t pos = offsets[blockIdx.x] + (uint32_t)block_exclusive_scan(__popc(fl), &total);
  const int D = d + 1;
  for (int u = 0; u < kItems; ++u) {
    if (!((fl >> u) & 1u)) continue;
    if ((int64_t)pos >= m) {  // the two counting passes disagree: never expected
      atomicOr(flags, BF_COLLISION);
      break;
    }
    const int64_t e = base + u;
    const int64_t i = e / D;
    const int k = (int)(e - i * D);
    for (int l = 0; l < d; ++l) keys[(int64_t)pos * d + l] = vertex_coord(pt_r0, pt_rank, i, d, k, l);
    tab_first[slot[e]] = kCanonBit | pos;
    ++pos;
  }
}

// Neighbour of lattice point j along direction k at offset t is
// key + t (1 - (d+1) e_k): +t on every stored coordinate except -t d on
// coordinate k (for k = d, +t on all of them). Thread g covers (k, j) with
// j fastest so that the writes to nbr[k][t][j] are contiguous.
__global__ __launch_bounds__(kBlock) void k_neighbors(const int32_t* __restrict__ keys, int64_t m,
                                                      int d, int r,
                                                      const unsigned long long* __restrict__ tab,
                                                      const uint32_t* __restrict__ tab_first,
                                                      unsigned long long mask,
                                                      HashCoef hc, unsigned long long maxp,
                                                      int32_t* __restrict__ nbr) {
  const int D = d + 1, T = 2 * r;
  const int64_t total = m * D;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) {
    const int k = (int)(g / m);
    const int64_t j = g - (int64_t)k * m;
    const int32_t* kj = keys + j * d;
    // offsets -t and +t together, so that the loads of both lookups are in
    // flight at once
    for (int t = 1; t <= r; ++t) {
      unsigned long long h[2] = {0, 0};
      for (int l = 0; l < d; ++l) {
        const int32_t c = kj[l];
        h[0] = hash_acc(h[0], hc.a[l], c + (l == k ? t * d : -t));
        h[1] = hash_acc(h[1], hc.a[l], c + (l == k ? -t * d : t));
      }
      int64_t sl[2];
      unsigned long long cur[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        h[u] = hash_final(h[u]);
        sl[u] = (int64_t)(h[u] & mask);
        cur[u] = tab[sl[u]];
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        // the first probe is usually decisive; otherwise keep probing
        if (cur[u] != h[u])
          sl[u] = cur[u] == kEmpty ? -1 : table_find_from(tab, mask, h[u], maxp, (unsigned long long)sl[u]);
      }
      uint32_t v[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) v[u] = sl[u] >= 0 ? tab_first[sl[u]] : 0u;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int tt = u == 0 ? -t : t;
        int32_t found = -1;
        const int64_t cand = (int64_t)(v[u] & ~kCanonBit);
        if (sl[u] >= 0 && (v[u] & kCanonBit) && cand < m) {
          bool same = true;
          for (int l = 0; l < d; ++l) same &= keys[cand * d + l] == kj[l] + (l == k ? -tt * d : tt);
          if (same) found = (int32_t)cand;
        }
        const int ti = tt < 0 ? tt + r : tt + r - 1;
        nbr[((int64_t)k * T + ti) * m + j] = found;
      }
    }
  }
}


// ---------------------------------------------------------------------------
// Internal order. Points are sorted by their remainder-0 lattice point
// (coordinates in units of d+1, packed most-significant-first into 64 bits,
// then the ranks of the first coordinates when they fit) so that a block of
// consecutive points touches few distinct lattice points;
// lattice points are then renumbered by first touch in that order, and W^T
// is stored as a CSR over those numbers so that the splat is a gather.

constexpr int kRankKey = 4;  // most coordinate ranks in the point sort key

struct KeyPack {
  int32_t lo[kMaxD];
  int32_t shift[kMaxD];
  int nk;  // leading dimensions packed into the key
  int nr;  // ranks of coordinates 0 .. nr-1 packed below them, rb bits each
  int rb;
};

__global__ __launch_bounds__(kBlock) void k_point_key(const int32_t* __restrict__ pt_r0,
                                                      const uint8_t* __restrict__ pt_rank, int64_t n, int d,
                                                      KeyPack kp, unsigned long long* __restrict__ key,
                                                      uint32_t* __restrict__ val) {
  const int D = d + 1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    unsigned long long k = 0;
    for (int l = 0; l < kp.nk; ++l)
      k |= (unsigned long long)(uint32_t)(pt_r0[i * d + l] / D - kp.lo[l]) << kp.shift[l];
    for (int l = 0; l < kp.nr; ++l)
      k |= (unsigned long long)pt_rank[i * d + l] << (kp.rb * (kp.nr - 1 - l));
    key[i] = k;
    val[i] = (uint32_t)i;
  }
}

__global__ __launch_bounds__(kBlock) void k_compact_internal(const uint32_t* __restrict__ bits,
                                                             const int32_t* __restrict__ slot_s,
                                                             uint32_t* __restrict__ first2, int64_t L,
                                                             const uint32_t* __restrict__ offsets,
                                                             const uint32_t* __restrict__ tab_first,
                                                             int64_t m, int32_t* __restrict__ int2can,
                                                             uint32_t* __restrict__ flags) {
  const int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)threadIdx.x * kItems;
  const uint32_t fl = base < L ? first_flags(bits, base) : 0u;
  int total;
  uint32_t pos = offsets[blockIdx.x] + (uint32_t)block_exclusive_scan(__popc(fl), &total);
  for (int u = 0; u < kItems; ++u) {
    if (!((fl >> u) & 1u)) continue;
    if ((int64_t)pos >= m) {
      atomicOr(flags, BF_COLLISION);
      break;
    }
    const int32_t sl = slot_s[base + u];
    int2can[pos] = (int32_t)(tab_first[sl] & ~kCanonBit);
    first2[sl] = kCanonBit | pos;
    ++pos;
  }
}

// (internal vertex, weight) of every (sorted point, vertex) element.
__global__ __launch_bounds__(kBlock) void k_resolve_internal(const int32_t* __restrict__ slot_s,
                                                             const uint32_t* __restrict__ first2,
                                                             const uint32_t* __restrict__ perm,
                                                             const float* __restrict__ w_orig,
                                                             int64_t L, int D, int64_t m,
                                                             sgp_entry* __restrict__ pm,
                                                             uint32_t* __restrict__ flags) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < L; e += stride) {
    const uint32_t v = first2[slot_s[e]];
    int32_t j = (int32_t)(v & ~kCanonBit);
    if (!(v & kCanonBit) || j >= m) {
      atomicOr(flags, BF_COLLISION);
      j = 0;
    }
    const int64_t ip = e / D;
    const int k = (int)(e - ip * D);
    sgp_entry en;
    en.j = j;
    en.w = w_orig[(int64_t)perm[ip] * D + k];
    pm[e] = en;
  }
}

__global__ __launch_bounds__(kBlock) void k_can2int(const int32_t* __restrict__ int2can, int64_t m,
                                                    int32_t* __restrict__ can2int) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += stride)
    can2int[int2can[j]] = (int32_t)j;
}

// Neighbour table in internal numbering: rows and entries both mapped, and
// laid out [direction][point][offset], so that the 2r neighbours of a point
// along one direction are adjacent (one 8-byte load for r = 1) in the blur.
// The canonical table is [direction][offset][point].
__global__ __launch_bounds__(kBlock) void k_nbr_internal(const int32_t* __restrict__ nbr_can,
                                                         const int32_t* __restrict__ int2can,
                                                         const int32_t* __restrict__ can2int,
                                                         int64_t m, int64_t D, int T,
                                                         int32_t* __restrict__ nbr_int) {
  const int64_t total = D * m * T;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) {
    const int64_t k = g / (m * T);
    const int64_t rest = g - k * m * T;
    const int64_t j = rest / T;
    const int64_t ti = rest - j * T;
    const int32_t nb = nbr_can[(k * T + ti) * m + int2can[j]];
    nbr_int[g] = nb >= 0 ? can2int[nb] : -1;
  }
}

// ---------------------------------------------------------------------------
// Tiles of P consecutive sorted points. Within a tile, entries are ordered by
// (internal lattice point, entry): equal lattice points form a "run" (one
// lattice point of one tile, its entries in sorted-point order), and runs are
// cut into pieces of at most K entries for the splat. A tile holds at most
// kTileSlots entries, so one block sorts it in LDS (a stable radix sort of
// the keys (lattice point << 12) | entry by lattice point), which gives the
// same order as a stable sort of all entries by (tile, lattice point).
constexpr int kTileThreads = 1024;
constexpr int kTileSlots = 4096;
constexpr int kTileSpan = kTileSlots / kTileThreads;  // consecutive slots per thread

// Thread t owns sorted positions 4t .. 4t+3; position i is kept at LDS
// index tile_at(i), so that the positions lanes access together are
// consecutive words (no bank conflicts).
__device__ __forceinline__ int tile_at(int i) { return (i & (kTileSpan - 1)) * kTileThreads + (i >> 2); }

struct TileSort {
  unsigned long long key[kTileSlots];  // at tile_at(position)
  int32_t rstart[kTileSlots];  // sorted position of each run's first entry (first the radix counters)
  int32_t wsum[kTileThreads / 64];
};

// Block-wide exclusive scan of one count per thread; *total gets the sum.
__device__ inline int tile_scan(int v, int32_t* wsum, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int before = 0, all = 0;
  for (int i = 0; i < kTileThreads / 64; ++i) {
    const int c = wsum[i];
    before += i < w ? c : 0;
    all += c;
  }
  __syncthreads();
  *total = all;
  return before + x - v;
}

// Stable LSD radix sort of all kTileSlots keys by their lattice-point field
// (key >> 12; entries past the tile hold ~0 and stay last), kRadixBits bits
// per pass. In a pass thread t holds positions t + u * kTileThreads (rounds
// u = 0..3). A key's rank among the keys of its wave and round with the
// same digit comes from the lanes' ballots of the digit bits; the counts
// per (digit, round, wave), scanned in that order, give every group its
// first position, so keys with equal digits keep their order. key[] holds
// the keys in entry order at tile_at(entry) on entry and the sorted keys
// at tile_at(position) on exit; hist takes kTileSlots counters.
constexpr int kRadixBits = 6;
static_assert((1 << kRadixBits) * kTileSpan * (kTileThreads / 64) == kTileSlots, "radix counters");
__device__ inline void tile_radix(unsigned long long* key, int32_t* hist, int32_t* wsum, int bits) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const unsigned long long below = (1ull << lane) - 1;
  unsigned long long v[kTileSpan];
#pragma unroll
  for (int u = 0; u < kTileSpan; ++u) v[u] = key[tile_at(t + u * kTileThreads)];
  for (int b = 0; b < bits; b += kRadixBits) {
    const int nb = bits - b < kRadixBits ? bits - b : kRadixBits;
    const bool last = b + nb >= bits;
#pragma unroll
    for (int k = 0; k < kTileSpan; ++k) hist[t * kTileSpan + k] = 0;
    __syncthreads();
    int dg[kTileSpan], rk[kTileSpan];
#pragma unroll
    for (int u = 0; u < kTileSpan; ++u) {
      dg[u] = (int)((v[u] >> (12 + b)) & ((1u << nb) - 1));
      unsigned long long peers = ~0ull;  // lanes whose digit equals this lane's
#pragma unroll
      for (int k = 0; k < kRadixBits; ++k) {
        if (k < nb) {
          const bool set = (dg[u] >> k) & 1;
          const unsigned long long bal = __ballot(set);
          peers &= set ? bal : ~bal;
        }
      }
      rk[u] = (int)__popcll(peers & below);
      if (rk[u] == 0) hist[(dg[u] * kTileSpan + u) * (kTileThreads / 64) + w] = (int)__popcll(peers);
    }
    __syncthreads();
    int h[kTileSpan], sum = 0;
#pragma unroll
    for (int k = 0; k < kTileSpan; ++k) {
      h[k] = hist[t * kTileSpan + k];
      sum += h[k];
    }
    int tot;
    int pre = tile_scan(sum, wsum, &tot);  // every thread has read its counters
#pragma unroll
    for (int k = 0; k < kTileSpan; ++k) {
      hist[t * kTileSpan + k] = pre;
      pre += h[k];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kTileSpan; ++u) {
      const int pos = hist[(dg[u] * kTileSpan + u) * (kTileThreads / 64) + w] + rk[u];
      key[last ? tile_at(pos) : pos] = v[u];
    }
    __syncthreads();
    if (!last) {
#pragma unroll
      for (int u = 0; u < kTileSpan; ++u) v[u] = key[t + u * kTileThreads];
    }
  }
}

// Run and piece starts of this thread's kTileSpan sorted positions, and
// their ranks within the tile. key[] holds the tile's sorted keys.
struct TileRanks {
  int q[kTileSpan];   // run of each position
  int qp[kTileSpan];  // piece of each position, where it starts one (else -1)
  bool rs[kTileSpan];
  int runs, pieces;
};
__device__ inline void tile_ranks(TileSort& T, int ne, int K, TileRanks& r) {
  const int i0 = threadIdx.x * kTileSpan;
  int c = 0;
#pragma unroll
  for (int u = 0; u < kTileSpan; ++u) {
    const int i = i0 + u;
    r.rs[u] = i < ne && (i == 0 || (T.key[tile_at(i)] >> 12) != (T.key[tile_at(i - 1)] >> 12));
    c += r.rs[u] ? 1 : 0;
  }
  int q = tile_scan(c, T.wsum, &r.runs) - 1;
#pragma unroll
  for (int u = 0; u < kTileSpan; ++u) {
    q += r.rs[u] ? 1 : 0;
    r.q[u] = q;
    if (r.rs[u]) T.rstart[q] = i0 + u;
  }
  __syncthreads();
  bool ps[kTileSpan];
  c = 0;
#pragma unroll
  for (int u = 0; u < kTileSpan; ++u) {
    const int i = i0 + u;
    ps[u] = i < ne && (i - T.rstart[r.q[u]]) % K == 0;
    c += ps[u] ? 1 : 0;
  }
  int qp = tile_scan(c, T.wsum, &r.pieces);
#pragma unroll
  for (int u = 0; u < kTileSpan; ++u) {
    r.qp[u] = ps[u] ? qp : -1;
    qp += ps[u] ? 1 : 0;
  }
}

// Pass 1: sort each tile, keep the order (entry within the tile per sorted
// position) and count its runs and pieces.
// Keys are also compared with their lattice point's canonical key (each
// run's first entry and each hashing group's first entry in a run):
// distinct keys with equal hashes in different groups share a lattice
// point, and one of those entries then differs from it.
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_tile_order(const sgp_entry* __restrict__ pm, int64_t n,
                                                             int D, int P, int K, int mbits, int Pi,
                                                             const uint32_t* __restrict__ perm,
                                                             const int32_t* __restrict__ pt_r0,
                                                             const uint8_t* __restrict__ pt_rank,
                                                             const int32_t* __restrict__ keys,
                                                             const int32_t* __restrict__ int2can,
                                                             uint16_t* __restrict__ ord,
                                                             uint32_t* __restrict__ runs,
                                                             uint32_t* __restrict__ pieces,
                                                             uint32_t* __restrict__ flags) {
  __shared__ TileSort T;
  const int64_t t = blockIdx.x;
  const int64_t p0 = t * P;
  const int ne = (int)((n - p0 < P ? n - p0 : P) * D);
  const int64_t base = p0 * D;
#pragma unroll
  for (int u = 0; u < kTileSpan; ++u) {
    const int i = threadIdx.x * kTileSpan + u;
    T.key[tile_at(i)] = i < ne ? ((unsigned long long)(uint32_t)pm[base + i].j << 12) | (unsigned)i : ~0ull;
  }
  __syncthreads();
  tile_radix(T.key, T.rstart, T.wsum, mbits);  // rstart is free until the ranks
  TileRanks r;
  tile_ranks(T, ne, K, r);
  // Positions whose key is compared with the stored key: the first entry of
  // each run, and within a run the first entry from each hashing group (the
  // blocks of k_tile_insert hold Pi sorted points and need not line up with
  // tiles; inside one group every entry already matched its group's first).
  // The run starts are no longer read, so their array takes the list.
  // A tile of P <= 3 Pi points meets at most three group starts; gs[]
  // holds them as entry indices within the tile (past the tile: never met).
  int gs[3];
  {
    const int off = (int)(p0 % Pi);  // points of the tile's first group before the tile
#pragma unroll
    for (int k = 0; k < 3; ++k) gs[k] = ((k + 1) * Pi - off) * D;
  }
  auto group_of = [&](int e) { return (e >= gs[0] ? 1 : 0) + (e >= gs[1] ? 1 : 0) + (e >= gs[2] ? 1 : 0); };
  bool ck[kTileSpan];
  int c = 0;
#pragma unroll
  for (int u = 0; u < kTileSpan; ++u) {
    const int i = threadIdx.x * kTileSpan + u;
    ck[u] = false;
    if (i < ne) {
      if (r.rs[u]) {
        ck[u] = true;
      } else {
        const int e = (int)(T.key[tile_at(i)] & 4095u);
        const int ep = (int)(T.key[tile_at(i - 1)] & 4095u);
        ck[u] = group_of(e) != group_of(ep);
      }
    }
    c += ck[u] ? 1 : 0;
  }
  int nchk;
  int pos = tile_scan(c, T.wsum, &nchk);
#pragma unroll
  for (int u = 0; u < kTileSpan; ++u)
    if (ck[u]) T.rstart[pos++] = threadIdx.x * kTileSpan + u;
  __syncthreads();
  const int d = D - 1;
  bool bad = false;
  for (int q = threadIdx.x; q < nchk; q += kTileThreads) {
    const unsigned long long k = T.key[tile_at(T.rstart[q])];
    const unsigned le = (unsigned)(k & 4095u);
    const int64_t pt = perm[p0 + le / (unsigned)D];
    const int kv = (int)(le % (unsigned)D);
    const int32_t* key = keys + (int64_t)int2can[k >> 12] * d;
    for (int l = 0; l < d; ++l) bad |= key[l] != vertex_coord(pt_r0, pt_rank, pt, d, kv, l);
  }
  if (bad) atomicOr(flags, BF_COLLISION);
  bool stray = false;
#pragma unroll
  for (int u = 0; u < kTileSpan; ++u) {
    const int i = threadIdx.x * kTileSpan + u;
    if (i < ne) {
      const int le = (int)(T.key[tile_at(i)] & 4095u);
      stray |= le >= ne;
      ord[base + i] = (uint16_t)(le < ne ? le : 0);  // never send the next pass past the tile
    }
  }
  if (stray) atomicOr(flags, BF_ORDER);
  if (threadIdx.x == 0) {
    runs[t] = (uint32_t)r.runs;
    pieces[t] = (uint32_t)r.pieces;
  }
}

// Pass 2, with each tile's first run and piece known: the slice's runs
// (lattice point per run, run slot per entry in point order), the splat's
// entries in run order (point within the tile, weight) and its pieces
// (first entry relative to the tile, lattice point).
__global__ __launch_bounds__(kTileThreads) void k_tile_fill(const sgp_entry* __restrict__ pm,
                                                            const uint16_t* __restrict__ ord, int64_t n,
                                                            int D, int P, int K,
                                                            const int32_t* __restrict__ tile_off,
                                                            const int32_t* __restrict__ stile_off,
                                                            int32_t* __restrict__ tile_verts,
                                                            uint16_t* __restrict__ loc,
                                                            float* __restrict__ ws,
                                                            uint8_t* __restrict__ ent_lp,
                                                            float* __restrict__ ent_w,
                                                            uint16_t* __restrict__ run_rel,
                                                            int32_t* __restrict__ piece_vert) {
  __shared__ TileSort T;
  const int64_t t = blockIdx.x;
  const int64_t p0 = t * P;
  const int ne = (int)((n - p0 < P ? n - p0 : P) * D);
  const int64_t base = p0 * D;
#pragma unroll
  for (int u = 0; u < kTileSpan; ++u) {
    const int i = threadIdx.x * kTileSpan + u;
    if (i >= ne) break;
    const unsigned le = ord[base + i];
    T.key[tile_at(i)] = ((unsigned long long)(uint32_t)pm[base + le].j << 12) | le;
    ws[base + i] = pm[base + i].w;
  }
  __syncthreads();
  TileRanks r;
  tile_ranks(T, ne, K, r);
  const int64_t q0 = tile_off[t], qp0 = stile_off[t];
  const int i0 = threadIdx.x * kTileSpan;
#pragma unroll
  for (int u = 0; u < kTileSpan; ++u) {
    const int i = i0 + u;
    if (i >= ne) break;
    const unsigned long long k = T.key[tile_at(i)];
    const int32_t j = (int32_t)(k >> 12);
    const unsigned le = (unsigned)(k & 4095u);
    ent_lp[base + i] = (uint8_t)(le / (unsigned)D);
    ent_w[base + i] = pm[base + le].w;
    loc[base + le] = (uint16_t)r.q[u];
    if (r.rs[u]) tile_verts[q0 + r.q[u]] = j;
    if (r.qp[u] >= 0) {
      run_rel[qp0 + r.qp[u]] = (uint16_t)i;
      piece_vert[qp0 + r.qp[u]] = j;
    }
  }
}

// Hashing and first occurrences, one group of kInsEntries / (d+1)
// consecutive sorted points per block. Its entries (simplex vertices) are
// hashed from the staged remainder-0 coordinates and ranks and grouped by
// hash in an LDS table whose slot keeps the group's smallest entry (its
// representative). The group is smaller than a tile, so that several blocks
// share a CU and hide each other's latencies. Each group is inserted
// into the global table once; per global slot the smallest caller-order
// entry (canonical numbering) and the smallest sorted-order entry (first
// touch) are kept with one atomic each per (tile, slot). Every entry's key
// must equal its representative's; one that differs is a hash collision.
constexpr int kInsThreads = 512;
constexpr int kInsSpan = 4;                          // consecutive entries per thread
constexpr int kInsEntries = kInsThreads * kInsSpan;  // entries per block, at most
constexpr int kInsTable = 2 * kInsEntries;           // LDS table slots (load factor <= 1/2)
constexpr uint32_t kLdsEmpty = 0xffffffffu;
struct TileInsertLds {
  unsigned long long h[kInsEntries];  // entry hashes; then (global slot, min caller entry) per representative
  uint32_t table[kInsTable];          // representative of the group in each slot
  int32_t r0[kInsEntries];            // the points' remainder-0 coordinates (points * d < kInsEntries)
  uint8_t rk[kInsEntries];            // and their ranks
  uint32_t op[kInsEntries / 2];       // caller index of each point
};

__device__ __forceinline__ int32_t staged_coord(const TileInsertLds& S, int lp, int d, int k, int l) {
  return S.r0[lp * d + l] + k - ((int)S.rk[lp * d + l] > d - k ? d + 1 : 0);
}

// Global slot of hash h: claimed by compare-and-swap if empty; -1 if full.
__device__ int64_t table_claim(unsigned long long* tab, unsigned long long mask, unsigned long long h,
                               unsigned long long maxp) {
  unsigned long long s = h & mask;
  for (unsigned long long probe = 0; probe <= mask && probe < maxp; ++probe) {
    const unsigned long long prev = atomicCAS(&tab[s], kEmpty, h);
    if (prev == kEmpty || prev == h) return (int64_t)s;
    s = (s + 1) & mask;
  }
  return -1;
}

__global__ __launch_bounds__(kInsThreads) void k_tile_insert(
    const uint32_t* __restrict__ perm, const int32_t* __restrict__ pt_r0,
    const uint8_t* __restrict__ pt_rank, int64_t n, int d, int P, unsigned long long* __restrict__ tab,
    uint32_t* __restrict__ tab_first, uint32_t* __restrict__ first2, unsigned long long mask,
    HashCoef hc, unsigned long long maxp, int32_t* __restrict__ slot, int32_t* __restrict__ slot_s,
    uint32_t* __restrict__ flags) {
  __shared__ TileInsertLds S;
  const int D = d + 1;
  const int64_t t = blockIdx.x;
  const int64_t p0 = t * P;
  const int np = (int)(n - p0 < P ? n - p0 : P);
  const int ne = np * D;
  const int64_t base = p0 * D;
  for (int lp = threadIdx.x; lp < np; lp += kInsThreads) S.op[lp] = perm[p0 + lp];
  for (int q = threadIdx.x; q < kInsTable; q += kInsThreads) S.table[q] = kLdsEmpty;
  __syncthreads();
  for (int q = threadIdx.x; q < np * d; q += kInsThreads) {
    const int lp = q / d, l = q - lp * d;
    const int64_t src = (int64_t)S.op[lp] * d + l;
    S.r0[q] = pt_r0[src];
    S.rk[q] = pt_rank[src];
  }
  __syncthreads();
  // thread tid owns entries e0 .. e0 + kInsSpan - 1
  const int e0 = threadIdx.x * kInsSpan;
  unsigned long long hv[kInsSpan];
#pragma unroll
  for (int u = 0; u < kInsSpan; ++u) {
    const int e = e0 + u;
    hv[u] = 0;
    if (e < ne) {
      const int lp = e / D, k = e - lp * D;
      unsigned long long h = 0;
      for (int l = 0; l < d; ++l) h = hash_acc(h, hc.a[l], staged_coord(S, lp, d, k, l));
      hv[u] = hash_final(h);
      S.h[e] = hv[u];
    }
  }
  __syncthreads();
  // group by hash: the first probe slot holding this hash, or an empty one
  // claimed; the slot then keeps the smallest entry of its group
  int ts[kInsSpan];
#pragma unroll
  for (int u = 0; u < kInsSpan; ++u) {
    const int e = e0 + u;
    ts[u] = -1;
    if (e >= ne) continue;
    int s = (int)(hv[u] & (kInsTable - 1));
    for (int probe = 0; probe < kInsTable; ++probe) {
      uint32_t cur = S.table[s];
      if (cur == kLdsEmpty) {
        cur = atomicCAS(&S.table[s], kLdsEmpty, (uint32_t)e);
        if (cur == kLdsEmpty) {
          ts[u] = s;
          break;
        }
      }
      if (S.h[cur] == hv[u]) {
        atomicMin(&S.table[s], (uint32_t)e);
        ts[u] = s;
        break;
      }
      s = (s + 1) & (kInsTable - 1);
    }
  }
  __syncthreads();
  int rep[kInsSpan];
#pragma unroll
  for (int u = 0; u < kInsSpan; ++u) rep[u] = ts[u] >= 0 ? (int)S.table[ts[u]] : -1;
  __syncthreads();  // the hashes are no longer read: representatives take (slot, min caller entry)
  uint32_t* g32 = reinterpret_cast<uint32_t*>(S.h);
  // the representatives' first probes go out together; a slot taken by
  // another hash (rare) continues probing on its own
  unsigned long long prev[kInsSpan];
#pragma unroll
  for (int u = 0; u < kInsSpan; ++u)
    prev[u] = rep[u] == e0 + u ? atomicCAS(&tab[hv[u] & mask], kEmpty, hv[u]) : kEmpty;
#pragma unroll
  for (int u = 0; u < kInsSpan; ++u) {
    const int e = e0 + u;
    if (rep[u] != e) continue;
    int64_t sl = (int64_t)(hv[u] & mask);
    if (prev[u] != kEmpty && prev[u] != hv[u]) sl = table_claim(tab, mask, hv[u], maxp);
    if (sl < 0) atomicOr(flags, BF_TABLE_FULL);
    g32[2 * e] = (uint32_t)sl;
    g32[2 * e + 1] = 0xffffffffu;
  }
  __syncthreads();
  bool bad = false;
  uint32_t eo[kInsSpan];
#pragma unroll
  for (int u = 0; u < kInsSpan; ++u) {
    const int e = e0 + u;
    if (rep[u] < 0) continue;
    const int lp = e / D, k = e - lp * D;
    eo[u] = S.op[lp] * (uint32_t)D + (uint32_t)k;  // caller-order entry
    atomicMin(&g32[2 * rep[u] + 1], eo[u]);
    const int rlp = rep[u] / D, rk = rep[u] - rlp * D;
    for (int l = 0; l < d; ++l) bad |= staged_coord(S, lp, d, k, l) != staged_coord(S, rlp, d, rk, l);
  }
  if (bad) atomicOr(flags, BF_COLLISION);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kInsSpan; ++u) {
    const int e = e0 + u;
    if (rep[u] < 0) continue;
    const int32_t sl = (int32_t)g32[2 * rep[u]];
    slot_s[base + e] = sl;
    slot[eo[u]] = sl;
    if (rep[u] == e && sl >= 0) {
      atomicMin(&tab_first[sl], g32[2 * e + 1]);
      atomicMin(&first2[sl], (uint32_t)(base + e));
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_occ_keys(const int32_t* __restrict__ vert, int64_t Q,
                                                     uint32_t* __restrict__ key,
                                                     uint32_t* __restrict__ val) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < Q; q += stride) {
    key[q] = (uint32_t)vert[q];
    val[q] = (uint32_t)q;
  }
}

// Pieces sorted (stably) by lattice point: row o of the splat's partial
// buffer belongs to piece val[o]; each lattice point's rows are contiguous.
__global__ __launch_bounds__(kBlock) void k_occ_fill(const uint32_t* __restrict__ key,
                                                     const uint32_t* __restrict__ val, int64_t Q,
                                                     int64_t m, int32_t* __restrict__ occ_ptr,
                                                     int32_t* __restrict__ run_dst,
                                                     int32_t* __restrict__ row_vert) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < Q; o += stride) {
    const uint32_t j = key[o];
    run_dst[val[o]] = (int32_t)o;
    row_vert[o] = (int32_t)j;
    if (o == 0 || key[o - 1] != j) occ_ptr[j] = (int32_t)o;
    if (o == Q - 1) occ_ptr[m] = (int32_t)Q;
  }
}

unsigned grid_for(int64_t work, int64_t per_block, int64_t cap) {
  int64_t b = (work + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

// Build temporaries. Once the stream has been synchronised after their last
// use (idle), they go back to the block cache; otherwise they are released
// in stream order.
struct Transient {
  static constexpr int kSlots = 24;
  void* ptr[kSlots] = {};
  size_t cap[kSlots] = {};
  hipStream_t s = nullptr;
  bool idle = false;
  int alloc(int slot_i, size_t bytes) {
    if (!bytes) bytes = 16;
    if ((ptr[slot_i] = block_take(bytes, &cap[slot_i]))) return SGP_OK;
    cap[slot_i] = bytes;
    hipError_t e = pool_alloc(&ptr[slot_i], bytes, s);
    if (e != hipSuccess) {
      ptr[slot_i] = nullptr;
      (void)hipGetLastError();
      set_error("device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
      return e == hipErrorOutOfMemory ? SGP_ENOMEM : SGP_EHIP;
    }
    return SGP_OK;
  }
  ~Transient() {
    for (int i = 0; i < kSlots; ++i) {
      if (!ptr[i]) continue;
      if (idle)
        block_give(ptr[i], cap[i]);
      else
        dev_release(ptr[i], s);
    }
  }
};

int bits_for(uint64_t range) {  // bits to hold values 0..range
  int b = 0;
  while (b < 64 && (range >> b) != 0) ++b;
  return b;
}

// shrink > 0 starts from a table 2^shrink times smaller than the bound
// L / load_factor (most lattices have far fewer distinct points than
// simplex vertices); *grow reports that it filled up, and the caller then
// repeats the attempt with the full table.
int build_attempt(sgp_lattice* L, const float* X, const double* f, double load_factor,
                  unsigned long long seed, int shrink, hipStream_t st, uint32_t* host_word, bool* retry,
                  bool* grow) {
  *retry = false;
  *grow = false;
  const int d = L->d, D = d + 1, T = 2 * L->order;
  const int64_t n = L->n;
  const int64_t Lel = n * D;
  int64_t cap = 1024;
  while ((double)cap * load_factor < (double)Lel) cap <<= 1;
  if (cap > (int64_t)1 << 31) {
    set_error("lattice_build: hash table of %lld slots exceeds 2^31; raise load_factor",
              (long long)cap);
    return SGP_EINVAL;
  }
  if (shrink > 0 && (cap >> shrink) >= 1024) cap >>= shrink;
  else shrink = 0;
  const unsigned long long maxp = shrink > 0 ? kMaxProbeReduced : kMaxProbe;
  const int64_t nb = (Lel + kChunk - 1) / kChunk;
  const HashCoef hc = hash_coef(seed);

  Transient tr;
  tr.s = st;
  int rc;
  enum {
    T_R0, T_RANK, T_SLOT, T_TAB, T_FIRST, T_COUNTS, T_OFFS, T_WORDS, T_W, T_NBRC,
    T_SLOTS, T_FIRST2, T_CAN2INT, T_KA, T_KB, T_VA, T_VB, T_SORTTMP, T_PM, T_SUB, T_ORD, T_CNT, T_BITS
  };
  if ((rc = tr.alloc(T_R0, sizeof(int32_t) * n * d))) return rc;
  if ((rc = tr.alloc(T_RANK, sizeof(uint8_t) * n * d))) return rc;
  if ((rc = tr.alloc(T_SLOT, sizeof(int32_t) * Lel))) return rc;
  if ((rc = tr.alloc(T_TAB, sizeof(unsigned long long) * cap))) return rc;
  if ((rc = tr.alloc(T_FIRST, sizeof(uint32_t) * cap))) return rc;
  if ((rc = tr.alloc(T_COUNTS, sizeof(uint32_t) * nb))) return rc;
  if ((rc = tr.alloc(T_OFFS, sizeof(uint32_t) * nb))) return rc;
  if ((rc = tr.alloc(T_WORDS, sizeof(uint32_t) * (4 + 2 * kMaxD)))) return rc;
  if ((rc = tr.alloc(T_W, sizeof(float) * Lel))) return rc;
  int32_t* pt_r0 = (int32_t*)tr.ptr[T_R0];
  uint8_t* pt_rank = (uint8_t*)tr.ptr[T_RANK];
  int32_t* slot = (int32_t*)tr.ptr[T_SLOT];
  unsigned long long* tab = (unsigned long long*)tr.ptr[T_TAB];
  uint32_t* tab_first = (uint32_t*)tr.ptr[T_FIRST];
  uint32_t* counts = (uint32_t*)tr.ptr[T_COUNTS];
  uint32_t* offs = (uint32_t*)tr.ptr[T_OFFS];
  uint32_t* words = (uint32_t*)tr.ptr[T_WORDS];  // [0] flags, [1] m, [2] m again, [4..] min/max
  float* w_orig = (float*)tr.ptr[T_W];
  int32_t* rmin = (int32_t*)(words + 4);
  int32_t* rmax = rmin + kMaxD;

  if ((rc = launch_fill_u32(words, 4, 0u, st))) return rc;
  if ((rc = launch_fill_u32((uint32_t*)rmin, kMaxD, 0x7fffffffu, st))) return rc;
  if ((rc = launch_fill_u32((uint32_t*)rmax, kMaxD, 0x80000000u, st))) return rc;

  SimplexArgs a;
  a.X = X;
  a.n = n;
  a.d = d;
  for (int j = 0; j < kMaxD; ++j) a.f[j] = j < d ? f[j] : 0.0;
  a.w = w_orig;
  a.pt_r0 = pt_r0;
  a.pt_rank = pt_rank;
  a.flags = words;
  a.rmin = rmin;
  a.rmax = rmax;
  {
    ProfScope ps(KK_SIMPLEX, st);
    hipLaunchKernelGGL(k_elevate, dim3(grid_for(n, kBlock / D, kElevateBlocks)), dim3(kBlock), 0, st, a);
    SGP_LAUNCH_CHECK("k_elevate");
  }
  const size_t nwords = 4 + 2 * kMaxD;
  SGP_HIP(hipMemcpyAsync(host_word, words, sizeof(uint32_t) * nwords, hipMemcpyDeviceToHost, st));
  SGP_HIP(hipStreamSynchronize(st));
  if (host_word[0] & BF_NONFINITE) {
    set_error("lattice_build: X contains NaN or Inf");
    return SGP_EINVAL;
  }
  if (host_word[0] & BF_OVERFLOW) {
    set_error("lattice_build: |x|/lengthscale too large, a lattice coordinate leaves int32");
    return SGP_EOVERFLOW;
  }
  // sort key: remainder-0 coordinates, leading dimensions first, as many as
  // fit in 64 bits; when all of them fit, the ranks of the first few
  // coordinates follow, so that points of one remainder-0 cell are grouped by
  // simplex and a tile touches fewer distinct lattice points
  KeyPack kp;
  int key_bits = 0;
  {
    const int32_t* hmin = (const int32_t*)(host_word + 4);
    const int32_t* hmax = hmin + kMaxD;
    int nk = 0, used = 0, bl[kMaxD];
    for (int l = 0; l < d; ++l) {
      const int b = bits_for((uint64_t)((int64_t)hmax[l] - (int64_t)hmin[l]));
      if (used + b > 64) break;
      bl[l] = b;
      used += b;
      nk = l + 1;
    }
    kp.nr = 0;
    kp.rb = bits_for((uint64_t)d);
    if (nk == d) kp.nr = std::min(std::min(d, kRankKey), (64 - used) / kp.rb);
    used += kp.nr * kp.rb;
    int sh = used;
    for (int l = 0; l < nk; ++l) {
      sh -= bl[l];
      kp.lo[l] = hmin[l];
      kp.shift[l] = sh;
    }
    kp.nk = nk;
    key_bits = used;
  }

  // ---- internal order: sort points, renumber vertices by first touch
  if ((rc = tr.alloc(T_SLOTS, sizeof(int32_t) * Lel))) return rc;
  if ((rc = tr.alloc(T_FIRST2, sizeof(uint32_t) * cap))) return rc;
  // sort buffers: 64-bit point keys (n), then 32-bit piece keys (at most Lel)
  const size_t kbytes = std::max(sizeof(unsigned long long) * n, sizeof(uint32_t) * Lel);
  if ((rc = tr.alloc(T_KA, kbytes))) return rc;
  if ((rc = tr.alloc(T_KB, kbytes))) return rc;
  if ((rc = tr.alloc(T_PM, sizeof(sgp_entry) * Lel))) return rc;
  if ((rc = tr.alloc(T_VA, sizeof(uint32_t) * Lel))) return rc;
  if ((rc = tr.alloc(T_VB, sizeof(uint32_t) * Lel))) return rc;
  if ((rc = tr.alloc(T_SORTTMP, sizeof(uint32_t) * radix_tmp_words(Lel)))) return rc;
  int32_t* slot_s = (int32_t*)tr.ptr[T_SLOTS];
  uint32_t* first2 = (uint32_t*)tr.ptr[T_FIRST2];
  uint32_t* va = (uint32_t*)tr.ptr[T_VA];
  uint32_t* vb = (uint32_t*)tr.ptr[T_VB];
  uint32_t* sort_tmp = (uint32_t*)tr.ptr[T_SORTTMP];
  for (sgp::DevBuf* b : {&L->perm, &L->loc, &L->ws, &L->tile_off, &L->tile_verts, &L->run_rel,
                         &L->ent_lp, &L->ent_w, &L->occ_ptr, &L->run_dst, &L->row_vert, &L->stile_off, &L->nbr, &L->int2can})
    dev_free(*b);
  if ((rc = dev_alloc(L->perm, sizeof(uint32_t) * n, st))) return rc;
  // two spare slots: the slice reads slots in aligned pairs
  if ((rc = dev_alloc(L->loc, sizeof(uint16_t) * (Lel + 2), st))) return rc;
  if ((rc = dev_alloc(L->ws, sizeof(float) * Lel, st))) return rc;
  sgp_entry* pm = (sgp_entry*)tr.ptr[T_PM];
  uint32_t* perm = (uint32_t*)L->perm.ptr;
  {
    unsigned long long* ka = (unsigned long long*)tr.ptr[T_KA];
    unsigned long long* kb = (unsigned long long*)tr.ptr[T_KB];
    {
      ProfScope ps(KK_ORDER, st);
      hipLaunchKernelGGL(k_point_key, dim3(grid_for(n, kBlock, 16384)), dim3(kBlock), 0, st, pt_r0,
                         (const uint8_t*)pt_rank, n, d, kp, ka, va);
      SGP_LAUNCH_CHECK("k_point_key");
    }
    bool in_alt = false;
    if ((rc = radix_sort_pairs<unsigned long long>(ka, va, kb, vb, n, key_bits, sort_tmp, st, &in_alt)))
      return rc;
    SGP_HIP(hipMemcpyAsync(perm, in_alt ? vb : va, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st));
  }
  // ---- hash the simplex vertices tile by tile in sorted order: slots, and
  // per slot the first entry in caller order and in sorted order
  // tile size: at most 256 points (a point index fits 8 bits) and 4096
  // entries (the tile kernels stage a tile's entries in LDS); a multiple of
  // 4, so that every tile's entries start 4-byte aligned in the 8- and
  // 16-bit arrays. (Smaller tiles for small inputs were measured and not
  // kept: a tile kernel's time on few tiles is the latency of one tile,
  // whatever its size, and the slice, one block per CU, then takes several
  // tiles per block.)
  const int P = std::min(256, 4096 / D) & ~3;
  if (P > 3 * (kInsEntries / D)) {  // k_tile_order follows at most three hashing groups per tile
    set_error("lattice_build: internal tile shape error (d = %d)", d);
    return SGP_EINVAL;
  }
  const int64_t ntiles = (n + P - 1) / P;
  if ((rc = launch_fill_u32((uint32_t*)tab, (size_t)cap * 2, 0u, st))) return rc;
  if ((rc = launch_fill_u32(tab_first, (size_t)cap, kNoFirst, st))) return rc;
  if ((rc = launch_fill_u32(first2, (size_t)cap, kNoFirst, st))) return rc;
  {
    ProfScope ps(KK_SIMPLEX, st);
    const int Pi = kInsEntries / D;
    hipLaunchKernelGGL(k_tile_insert, dim3((unsigned)((n + Pi - 1) / Pi)), dim3(kInsThreads), 0, st,
                       (const uint32_t*)perm, (const int32_t*)pt_r0, (const uint8_t*)pt_rank, n, d, Pi, tab,
                       tab_first, first2, (unsigned long long)(cap - 1), hc, maxp, slot, slot_s, words);
    SGP_LAUNCH_CHECK("k_tile_insert");
  }
  // first-occurrence bitmasks: caller order (canonical numbering), sorted order (first touch)
  const int64_t nwords_bits = (Lel + 31) / 32;
  if ((rc = tr.alloc(T_BITS, sizeof(uint32_t) * 2 * nwords_bits))) return rc;
  uint32_t* bits1 = (uint32_t*)tr.ptr[T_BITS];
  uint32_t* bits2 = bits1 + nwords_bits;
  if ((rc = launch_fill_u32(bits1, (size_t)(2 * nwords_bits), 0u, st))) return rc;
  {
    ProfScope ps(KK_COUNT, st);
    hipLaunchKernelGGL(k_mark_first, dim3(grid_for(cap, kBlock, 16384)), dim3(kBlock), 0, st,
                       (const uint32_t*)tab_first, cap, bits1);
    SGP_LAUNCH_CHECK("k_mark_first");
    hipLaunchKernelGGL(k_mark_first, dim3(grid_for(cap, kBlock, 16384)), dim3(kBlock), 0, st,
                       (const uint32_t*)first2, cap, bits2);
    SGP_LAUNCH_CHECK("k_mark_first");
    hipLaunchKernelGGL(k_count_first, dim3((unsigned)nb), dim3(kBlock), 0, st, (const uint32_t*)bits1, Lel,
                       counts);
    SGP_LAUNCH_CHECK("k_count_first");
  }
  {
    ProfScope ps(KK_SCAN, st);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, st, counts, offs, nb, words + 1);
    SGP_LAUNCH_CHECK("k_scan");
  }
  SGP_HIP(hipMemcpyAsync(host_word, words, sizeof(uint32_t) * 2, hipMemcpyDeviceToHost, st));
  SGP_HIP(hipStreamSynchronize(st));
  const uint32_t flags = host_word[0];
  const int64_t m = host_word[1];
  if (flags & BF_TABLE_FULL) {
    if (shrink > 0) {  // the reduced table was too small: repeat with the full one
      tr.idle = true;
      *grow = true;
      return SGP_OK;
    }
    set_error("lattice_build: hash table full");
    return SGP_EHASH;
  }
  if (flags & BF_COLLISION) {  // two keys share a 64-bit hash: try another seed
    tr.idle = true;
    *retry = true;
    return SGP_OK;
  }
  if (m < 1 || m > Lel) {
    set_error("lattice_build: inconsistent lattice size %lld", (long long)m);
    return SGP_EHASH;
  }
  L->m = m;
  dev_free(L->keys);
  if ((rc = dev_alloc(L->keys, sizeof(int32_t) * m * d, st))) return rc;
  if ((rc = dev_alloc(L->nbr, sizeof(int32_t) * m * D * T, st))) return rc;
  if ((rc = dev_alloc(L->int2can, sizeof(int32_t) * m, st))) return rc;
  if ((rc = tr.alloc(T_NBRC, sizeof(int32_t) * m * D * T))) return rc;
  if ((rc = tr.alloc(T_CAN2INT, sizeof(int32_t) * m))) return rc;
  int32_t* nbr_can = (int32_t*)tr.ptr[T_NBRC];
  int32_t* can2int = (int32_t*)tr.ptr[T_CAN2INT];
  {
    ProfScope ps(KK_COMPACT, st);
    hipLaunchKernelGGL(k_compact, dim3((unsigned)nb), dim3(kBlock), 0, st, (const uint32_t*)bits1, slot,
                       tab_first, Lel, offs,
                       pt_r0, pt_rank, d, m, (int32_t*)L->keys.ptr, words);
    SGP_LAUNCH_CHECK("k_compact");
  }
  {
    ProfScope ps(KK_NEIGHBORS, st);
    hipLaunchKernelGGL(k_neighbors, dim3(grid_for(m * D, kBlock, 16384)), dim3(kBlock), 0, st,
                       (const int32_t*)L->keys.ptr, m, d, L->order, tab, tab_first,
                       (unsigned long long)(cap - 1), hc, maxp, nbr_can);
    SGP_LAUNCH_CHECK("k_neighbors");
  }
  // ---- internal numbering: lattice points by first touch in sorted order
  {
    ProfScope ps(KK_COUNT, st);
    hipLaunchKernelGGL(k_count_first, dim3((unsigned)nb), dim3(kBlock), 0, st, (const uint32_t*)bits2, Lel,
                       counts);
    SGP_LAUNCH_CHECK("k_count_first");
  }
  {
    ProfScope ps(KK_SCAN, st);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, st, counts, offs, nb, words + 2);
    SGP_LAUNCH_CHECK("k_scan");
  }
  {
    ProfScope ps(KK_ORDER, st);
    hipLaunchKernelGGL(k_compact_internal, dim3((unsigned)nb), dim3(kBlock), 0, st, (const uint32_t*)bits2,
                       slot_s, first2, Lel,
                       offs, tab_first, m, (int32_t*)L->int2can.ptr, words);
    SGP_LAUNCH_CHECK("k_compact_internal");
    hipLaunchKernelGGL(k_resolve_internal, dim3(grid_for(Lel, kBlock, 16384)), dim3(kBlock), 0, st,
                       slot_s, first2, perm, w_orig, Lel, D, m, pm, words);
    SGP_LAUNCH_CHECK("k_resolve_internal");
    hipLaunchKernelGGL(k_can2int, dim3(grid_for(m, kBlock, 16384)), dim3(kBlock), 0, st,
                       (const int32_t*)L->int2can.ptr, m, can2int);
    SGP_LAUNCH_CHECK("k_can2int");
    hipLaunchKernelGGL(k_nbr_internal, dim3(grid_for(m * D * T, kBlock, 16384)), dim3(kBlock), 0, st,
                       nbr_can, (const int32_t*)L->int2can.ptr, can2int, m, (int64_t)D, T,
                       (int32_t*)L->nbr.ptr);
    SGP_LAUNCH_CHECK("k_nbr_internal");
  }
  // ---- tiles of consecutive sorted points, their runs, and runs per lattice point
  {
    L->tile_points = P;
    L->ntiles = ntiles;
    const int mb = bits_for((uint64_t)(m - 1));
    if ((rc = tr.alloc(T_ORD, sizeof(uint16_t) * Lel))) return rc;
    if ((rc = tr.alloc(T_CNT, sizeof(uint32_t) * 2 * ntiles))) return rc;
    uint16_t* ord = (uint16_t*)tr.ptr[T_ORD];
    uint32_t* runs = (uint32_t*)tr.ptr[T_CNT];
    uint32_t* pieces = runs + ntiles;
    if ((rc = dev_alloc(L->tile_off, sizeof(int32_t) * (ntiles + 1), st))) return rc;
    if ((rc = dev_alloc(L->stile_off, sizeof(int32_t) * (ntiles + 1), st))) return rc;
    int32_t* tile_off = (int32_t*)L->tile_off.ptr;
    int32_t* stile_off = (int32_t*)L->stile_off.ptr;
    {
      ProfScope ps(KK_ORDER, st);
      hipLaunchKernelGGL(k_tile_order, dim3((unsigned)ntiles), dim3(kTileThreads), 0, st,
                         (const sgp_entry*)tr.ptr[T_PM], n, D, P, kPiece, mb, kInsEntries / D,
                         (const uint32_t*)perm,
                         (const int32_t*)pt_r0, (const uint8_t*)pt_rank, (const int32_t*)L->keys.ptr,
                         (const int32_t*)L->int2can.ptr, ord, runs, pieces, words);
      SGP_LAUNCH_CHECK("k_tile_order");
    }
    // first run and first piece of every tile; the totals land in entry ntiles
    if ((rc = scan_exclusive_u32(runs, (uint32_t*)tile_off, ntiles, (uint32_t*)tile_off + ntiles,
                                 sort_tmp, st)))
      return rc;
    if ((rc = scan_exclusive_u32(pieces, (uint32_t*)stile_off, ntiles, (uint32_t*)stile_off + ntiles,
                                 sort_tmp, st)))
      return rc;
    // longest run list and piece list of a tile (they size the LDS stages)
    std::vector<int32_t> toff(ntiles + 1), soff(ntiles + 1);
    SGP_HIP(hipMemcpyAsync(toff.data(), tile_off, sizeof(int32_t) * (ntiles + 1), hipMemcpyDeviceToHost, st));
    SGP_HIP(hipMemcpyAsync(soff.data(), stile_off, sizeof(int32_t) * (ntiles + 1), hipMemcpyDeviceToHost, st));
    SGP_HIP(hipStreamSynchronize(st));
    const int64_t Q = toff[ntiles], Qs = soff[ntiles];
    if (Q < 1 || Q > Lel || Qs < Q || Qs > Lel) {
      set_error("lattice_build: inconsistent run / piece counts %lld / %lld", (long long)Q, (long long)Qs);
      return SGP_EHASH;
    }
    int mx = 0, msx = 0;
    for (int64_t t = 0; t < ntiles; ++t) {
      mx = std::max(mx, toff[t + 1] - toff[t]);
      msx = std::max(msx, soff[t + 1] - soff[t]);
    }
    L->nrun = Q;
    L->npiece = Qs;
    L->max_tile_runs = mx;
    L->max_tile_pieces = msx;
    if ((rc = dev_alloc(L->tile_verts, sizeof(int32_t) * Q, st))) return rc;
    // four spare bytes: the splat reads entry points four at a time
    if ((rc = dev_alloc(L->ent_lp, sizeof(uint8_t) * (Lel + 4), st))) return rc;
    if ((rc = dev_alloc(L->ent_w, sizeof(float) * Lel, st))) return rc;
    if ((rc = dev_alloc(L->run_rel, sizeof(uint16_t) * Qs, st))) return rc;
    if ((rc = dev_alloc(L->occ_ptr, sizeof(int32_t) * (m + 1), st))) return rc;
    if ((rc = dev_alloc(L->run_dst, sizeof(int32_t) * Qs, st))) return rc;
    if ((rc = dev_alloc(L->row_vert, sizeof(int32_t) * Qs, st))) return rc;
    if ((rc = tr.alloc(T_SUB, sizeof(uint32_t) * Qs))) return rc;
    uint32_t* sub = (uint32_t*)tr.ptr[T_SUB];  // lattice point of each piece
    {
      ProfScope ps(KK_ORDER, st);
      hipLaunchKernelGGL(k_tile_fill, dim3((unsigned)ntiles), dim3(kTileThreads), 0, st,
                         (const sgp_entry*)tr.ptr[T_PM], (const uint16_t*)ord, n, D, P, kPiece,
                         (const int32_t*)tile_off, (const int32_t*)stile_off, (int32_t*)L->tile_verts.ptr,
                         (uint16_t*)L->loc.ptr, (float*)L->ws.ptr, (uint8_t*)L->ent_lp.ptr,
                         (float*)L->ent_w.ptr, (uint16_t*)L->run_rel.ptr, (int32_t*)sub);
      SGP_LAUNCH_CHECK("k_tile_fill");
    }
    // pieces grouped by lattice point (32-bit keys; reuses the sort buffers)
    uint32_t* k32a = (uint32_t*)tr.ptr[T_KA];
    uint32_t* k32b = (uint32_t*)tr.ptr[T_KB];
    {
      ProfScope ps(KK_ORDER, st);
      hipLaunchKernelGGL(k_occ_keys, dim3(grid_for(Qs, kBlock, 16384)), dim3(kBlock), 0, st,
                         (const int32_t*)sub, Qs, k32a, va);
      SGP_LAUNCH_CHECK("k_occ_keys");
    }
    bool occ_alt = false;
    if ((rc = radix_sort_pairs<uint32_t>(k32a, va, k32b, vb, Qs, mb, sort_tmp, st, &occ_alt))) return rc;
    {
      ProfScope ps(KK_ORDER, st);
      hipLaunchKernelGGL(k_occ_fill, dim3(grid_for(Qs, kBlock, 16384)), dim3(kBlock), 0, st,
                         occ_alt ? k32b : k32a, occ_alt ? vb : va, Qs, m, (int32_t*)L->occ_ptr.ptr,
                         (int32_t*)L->run_dst.ptr, (int32_t*)L->row_vert.ptr);
      SGP_LAUNCH_CHECK("k_occ_fill");
    }
  }
  SGP_HIP(hipMemcpyAsync(host_word, words, sizeof(uint32_t) * 3, hipMemcpyDeviceToHost, st));
  SGP_HIP(hipStreamSynchronize(st));
  tr.idle = true;  // every kernel of this attempt has finished
  if (host_word[0] & BF_ORDER) {
    set_error("lattice_build: internal error, a tile's sorted order is not a permutation");
    return SGP_EHASH;
  }
  if (host_word[0] & BF_COLLISION) *retry = true;
  if (!*retry && (int64_t)host_word[2] != m) {
    set_error("lattice_build: internal numbering found %u lattice points, expected %lld",
              host_word[2], (long long)m);
    return SGP_EHASH;
  }
  return SGP_OK;
}

}  // namespace
}  // namespace sgp

using namespace sgp;

// Hash-table shape of a build: the load factor bounding the full table
// (L / load_factor slots for L = n(d+1) splat entries) and the first
// attempt's reduction of it (2^shrink times smaller; a build whose table
// fills up repeats with the full one). Neither changes any result: lattice
// points are numbered by first occurrence, not by slot.
namespace sgp {
namespace {
struct BuildShape {
  float load_factor;
  int shrink;
};
struct BuildTuneEntry {
  int d, llog;
  BuildShape shape;
  float ms;
};
std::mutex g_build_tune_mu;
std::vector<BuildTuneEntry> g_build_tune;          // process-wide, keyed by (d, size class)
thread_local const BuildShape* g_build_force = nullptr;  // set while candidates are timed
constexpr BuildShape kDefaultShape{0.5f, 3};

int llog_of(int64_t L) {
  int b = 0;
  while (((int64_t)1 << b) < L) ++b;
  return b;
}

BuildShape build_shape(int64_t n, int d, float load_factor) {
  if (g_build_force) return *g_build_force;
  if (load_factor > 0.f) return BuildShape{load_factor, kDefaultShape.shrink};
  std::lock_guard<std::mutex> lk(g_build_tune_mu);
  for (const BuildTuneEntry& e : g_build_tune)
    if (e.d == d && e.llog == llog_of(n * (d + 1))) return e.shape;
  return kDefaultShape;
}
}  // namespace

void build_tune_reset() {
  std::lock_guard<std::mutex> lk(g_build_tune_mu);
  g_build_tune.clear();
}
}  // namespace sgp

extern "C" int lattice_build(const float* X, int64_t n, int32_t d, const double* lengthscales,
                             const sgp_opts* opts, void* stream, sgp_lattice** out) {
  if (!out) {
    set_error("lattice_build: out is NULL");
    return SGP_EINVAL;
  }
  *out = nullptr;
  sgp_opts o;
  sgp_opts_default(&o);
  if (opts) o = *opts;
  if (!X || !lengthscales) {
    set_error("lattice_build: X and lengthscales must be non-NULL");
    return SGP_EINVAL;
  }
  if (n < 1 || d < 1 || d > kMaxD) {
    set_error("lattice_build: need n >= 1 and 1 <= d <= %d (got n=%lld, d=%d)", kMaxD,
              (long long)n, (int)d);
    return SGP_EINVAL;
  }
  if (n > ((int64_t)1 << 30) / (d + 1)) {
    set_error("lattice_build: n*(d+1) must not exceed 2^30");
    return SGP_EINVAL;
  }
  for (int j = 0; j < d; ++j) {
    if (!(lengthscales[j] > 0.0) || !std::isfinite(lengthscales[j])) {
      set_error("lattice_build: lengthscale %d is not finite and positive", j);
      return SGP_EINVAL;
    }
  }
  if (o.order < 1 || o.order > kMaxOrder) {
    set_error("lattice_build: order must be in 1..%d", kMaxOrder);
    return SGP_EINVAL;
  }
  if (o.kernel != SGP_KERNEL_RBF && o.kernel != SGP_KERNEL_MATERN32) {
    set_error("lattice_build: unknown kernel %d", o.kernel);
    return SGP_EINVAL;
  }
  if (o.blur != SGP_BLUR_SYMMETRIC && o.blur != SGP_BLUR_FORWARD && o.blur != SGP_BLUR_REVERSE) {
    set_error("lattice_build: unknown blur order %d", o.blur);
    return SGP_EINVAL;
  }
  if (!std::isfinite(o.outputscale)) {
    set_error("lattice_build: outputscale must be finite");
    return SGP_EINVAL;
  }
  if (o.solve_rows < 0 || o.solve_rows > n) {
    set_error("lattice_build: solve_rows must be in [0, n]");
    return SGP_EINVAL;
  }
  if (!(o.load_factor == 0.0f || (o.load_factor > 0.0f && o.load_factor <= 0.9f))) {
    set_error("lattice_build: load_factor must be 0 (automatic) or in (0, 0.9]");
    return SGP_EINVAL;
  }
  const BuildShape shape = build_shape(n, d, o.load_factor);

  hipStream_t st = (hipStream_t)stream;
  sgp_lattice* L = new sgp_lattice();
  L->n = n;
  L->d = d;
  L->order = o.order;
  L->kernel = o.kernel;
  L->blur = o.blur;
  L->outputscale = o.outputscale;
  L->solve_rows = o.solve_rows;
  double f[kMaxD];
  make_constants(d, o.order, o.kernel, lengthscales, &L->spacing, L->stencil64, f);
  for (int j = 0; j < d; ++j) L->ell[j] = lengthscales[j];

  int rc = SGP_OK;
  uint32_t* host_word = (uint32_t*)pinned_scratch(sizeof(uint32_t) * (4 + 2 * kMaxD));
  {
    hipError_t e = hipGetDevice(&L->device);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&L->last_use, hipEventDisableTiming);
    if (e != hipSuccess) rc = hip_fail(e, "lattice_build setup", __FILE__, __LINE__);
    if (!host_word && rc == SGP_OK) {
      set_error("lattice_build: pinned host scratch unavailable");
      rc = SGP_ENOMEM;
    }
  }
  bool retry = true;
  int shrink = shape.shrink;  // first try a table 2^shrink times smaller than the bound
  for (int attempt = 0; rc == SGP_OK && retry && attempt < 4;) {
    const unsigned long long seed = 0x5157a11ce5eedull + 0x9e3779b97f4a7c15ull * (unsigned long long)attempt;
    bool grow = false;
    rc = build_attempt(L, X, f, (double)shape.load_factor, seed, shrink, st, host_word, &retry, &grow);
    if (rc == SGP_OK && grow) {
      shrink = 0;
      retry = true;
      continue;
    }
    ++attempt;
  }
  if (rc == SGP_OK && retry) {
    set_error("lattice_build: hash verification failed after 4 seeds");
    rc = SGP_EHASH;
  }
  if (rc == SGP_OK) {
    hipError_t e = hipStreamSynchronize(st);  // transient buffers are released on the stream
    if (e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize", __FILE__, __LINE__);
    mark_use(L, st);
  }
  if (rc != SGP_OK) {
    (void)hipStreamSynchronize(st);  // nothing may still use the buffers being released
    (void)hipGetLastError();
    lattice_free(L);
    return rc;
  }
  *out = L;
  return SGP_OK;
}

// Times lattice_build of X for every candidate hash-table shape and keeps
// the fastest for builds of the same d and size class.
extern "C" int sgp_autotune_build(const float* X, int64_t n, int32_t d, const double* lengthscales,
                                  const sgp_opts* opts, int32_t reps, void* stream, float* load_factor,
                                  int32_t* shrink, float* ms_per_build) {
  using namespace sgp;
  if (reps < 1) {
    set_error("sgp_autotune_build: reps must be >= 1");
    return SGP_EINVAL;
  }
  sgp_opts o;
  sgp_opts_default(&o);
  if (opts) o = *opts;
  o.load_factor = 0.f;
  static const BuildShape kCandidates[] = {{0.25f, 3}, {0.5f, 3}, {0.9f, 3}, {0.5f, 2}, {0.5f, 4},
                                           {0.5f, 0}, {0.9f, 0}};
  BuildShape best = kDefaultShape;
  float best_ms = -1.f;
  struct Reset {
    ~Reset() { g_build_force = nullptr; }
  } reset;
  for (const BuildShape& cand : kCandidates) {
    g_build_force = &cand;
    float ms = 0.f;
    for (int r = 0; r <= reps; ++r) {  // one warm-up, then reps timed builds
      sgp_lattice* L = nullptr;
      const auto t0 = std::chrono::steady_clock::now();
      const int rc = lattice_build(X, n, d, lengthscales, &o, stream, &L);
      const auto t1 = std::chrono::steady_clock::now();
      if (rc) return rc;
      lattice_free(L);
      if (r > 0) ms += std::chrono::duration<float, std::milli>(t1 - t0).count();
    }
    ms /= (float)reps;
    if (best_ms < 0.f || ms < best_ms) {
      best_ms = ms;
      best = cand;
    }
  }
  g_build_force = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_build_tune_mu);
    const BuildTuneEntry e{(int)d, llog_of(n * (d + 1)), best, best_ms};
    bool found = false;
    for (BuildTuneEntry& x : g_build_tune)
      if (x.d == e.d && x.llog == e.llog) {
        x = e;
        found = true;
      }
    if (!found) g_build_tune.push_back(e);
  }
  if (load_factor) *load_factor = best.load_factor;
  if (shrink) *shrink = best.shrink;
  if (ms_per_build) *ms_per_build = best_ms;
  return SGP_OK;
}
