// The lattice MVM  out = outputscale * W_X K_UU W_X^T V  (Section 4, eq. ski_to_bf).
//
// Everything runs in the lattice's internal order: points sorted by their
// remainder-0 lattice point, lattice points numbered by first touch in that
// order, sorted points cut into tiles of at most 256 points, and each tile
// carrying the ascending list of lattice points it touches (its runs).
//   k_splat_tile    W^T restricted to one tile: the tile's values are staged
//                   in LDS and every run sums its entries from there
//                   (Section 3.2, Splat), giving one partial row per run
//   k_splat_gather  U[j] = sum of the partial rows of lattice point j over
//                   the tiles that touch it
//   k_blur          one step of the blur along one lattice direction per
//                   chain: U'[j] = sum_t stencil[t] U[nbr(j, k, t)], missing
//                   neighbours contributing zero (Section 3.2, Blur). In
//                   SYMMETRIC order one thread advances the forward chain
//                   (direction step) and the reverse chain (direction d-step)
//                   of its row, and the last step stores their sum.
//   k_slice_tile    out = scale * W U: the tile's lattice rows are staged in
//                   LDS, every point combines its d+1 rows from there
//                   (Section 3.2, Slice); the CG variant adds noise * p and
//                   emits per-tile partial sums of p . out per column.
// Every sum runs in a fixed order: no atomics, results independent of
// scheduling. Values in the caller's point order are reached through the
// permutation (rows of V gathered when staged, rows of out scattered); the
// CG solver keeps its vectors in internal order and skips it.
//
// Channels are processed in chunks of G (a power of two <= 16) chosen so
// that the staged rows fit the LDS budget; chunks are the grid's y axis.
// Row ranges of consecutive blocks go to the same XCD (blocks are dealt
// round-robin over the 8 XCDs), so tiles that share lattice points share
// an L2.
#include <mutex>
#include <type_traits>
#include <vector>

#include "cg_step.h"
#include "sgp_internal.h"

namespace sgp {
namespace {

constexpr int kXcds = 8;

// Logical block for dispatch slot b when blocks are dealt round-robin over
// the XCDs: XCD x runs logical blocks [x*q + min(x, r), ...) contiguously.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t x = b % kXcds, t = b / kXcds;
  const int64_t q = nb / kXcds, r = nb % kXcds;
  return x * q + (x < r ? x : r) + t;
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// 16-byte vectors for LDS and global accesses of lattice and point rows.
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
  typedef dvec2 T;
  static constexpr int N = 2;
};
template <>
struct Vec16<float> {
  typedef fvec4 T;
  static constexpr int N = 4;
};

// Read (or write) W consecutive elements at p, as 16-byte vectors when W
// elements span whole vectors (p is then 16-byte aligned by construction).
template <typename T, int W>
__device__ __forceinline__ void read_row(const T* p, T (&o)[W]) {
  constexpr int N = Vec16<T>::N;
  if constexpr (W % N == 0) {
#pragma unroll
    for (int i = 0; i < W / N; ++i) {
      const typename Vec16<T>::T x = *(const typename Vec16<T>::T*)(p + i * N);
#pragma unroll
      for (int j = 0; j < N; ++j) o[i * N + j] = x[j];
    }
  } else {
#pragma unroll
    for (int i = 0; i < W; ++i) o[i] = p[i];
  }
}
template <typename T, int W>
__device__ __forceinline__ void write_row(T* p, const T (&v)[W]) {
  constexpr int N = Vec16<T>::N;
  if constexpr (W % N == 0) {
#pragma unroll
    for (int i = 0; i < W / N; ++i) {
      typename Vec16<T>::T x;
#pragma unroll
      for (int j = 0; j < N; ++j) x[j] = v[i * N + j];
      *(typename Vec16<T>::T*)(p + i * N) = x;
    }
  } else {
#pragma unroll
    for (int i = 0; i < W; ++i) p[i] = v[i];
  }
}

// read_row with non-temporal loads
template <typename T, int W>
__device__ __forceinline__ void read_row_nt(const T* p, T (&o)[W]) {
  constexpr int N = Vec16<T>::N;
  if constexpr (W % N == 0) {
#pragma unroll
    for (int i = 0; i < W / N; ++i) {
      const typename Vec16<T>::T x = __builtin_nontemporal_load((const typename Vec16<T>::T*)(p + i * N));
#pragma unroll
      for (int j = 0; j < N; ++j) o[i * N + j] = x[j];
    }
  } else {
#pragma unroll
    for (int i = 0; i < W; ++i) o[i] = __builtin_nontemporal_load(p + i);
  }
}

// write_row with non-temporal stores (streamed past the caches)
template <typename TU, int W>
__device__ __forceinline__ void write_row_nt(TU* p, const TU (&v)[W]) {
  constexpr int N = Vec16<TU>::N;
  if constexpr (W % N == 0) {
#pragma unroll
    for (int i = 0; i < W / N; ++i) {
      typename Vec16<TU>::T x;
#pragma unroll
      for (int j = 0; j < N; ++j) x[j] = v[i * N + j];
      __builtin_nontemporal_store(x, (typename Vec16<TU>::T*)(p + i * N));
    }
  } else {
#pragma unroll
    for (int i = 0; i < W; ++i) __builtin_nontemporal_store(v[i], p + i);
  }
}

// Persistent tile kernels: block b runs on XCD b % 8 and takes work items
// from a contiguous range owned by its XCD, striding over it with the other
// blocks of that XCD.
__device__ __forceinline__ void xcd_items(int64_t items, int64_t* first, int64_t* end, int64_t* step) {
  const int64_t nb = gridDim.x, b = blockIdx.x;
  const int64_t x = b % kXcds, k = b / kXcds;
  const int64_t per = nb / kXcds, rem = nb % kXcds;
  const int64_t before = x * per + (x < rem ? x : rem);
  const int64_t mine = per + (x < rem ? 1 : 0);
  const int64_t lo = items * before / nb;
  const int64_t hi = items * (before + mine) / nb;
  *first = lo + k;
  *end = hi;
  *step = mine;
}

// Per-thread register shapes of the tile kernels (NT threads per block, at
// most 256 points and kMaxTileEntries entries and runs per tile).
constexpr int kMaxTileEntries = 4096;
constexpr int kSplatBlock = 512;   // two blocks per CU
// The slice adds a point's entries by blocks of this many runs of its tile's
// run list; every staged chunk (at most 16 channels) holds a whole number of
// such blocks (RC = 8 NT / G >= 512).
constexpr int kSliceOrderRows = 512;
// Threads per block of k_slice_tile: 1024 (one block per CU), or for narrow
// channel chunks just the lane groups for the 256 points of a tile (LPR =
// G / VW lanes each), so that the lanes are not left idle. The narrow block
// also stages fewer lattice rows per pass (RC = 8 NT / G), so it is taken
// only where a tile's runs mostly fit in one pass.
template <int G>
constexpr int slice_threads_narrow() { return G >= 16 ? 1024 : G == 8 ? 512 : 256; }
template <typename TU, int G, int NT_>
struct TileShape {
  static constexpr int NT = NT_;
  static constexpr int kPts = 256;
  static constexpr int EPT = kMaxTileEntries / NT;  // entries per thread
  static constexpr int RPT = 2;                      // runs prefetched per thread (splat)
  static constexpr int VPT = (kPts * G) / NT > 0 ? (kPts * G) / NT : 1;  // point values
  static constexpr int VW = G < 4 ? G : 4;  // channels per lane
  static constexpr int LPR = G / VW;        // lanes per run (splat) or point (slice)
  static constexpr int NG = NT / LPR;
  static constexpr int UPT = 8;             // lattice rows staged per thread in the slice
  static constexpr int RC = UPT * NT / G;   // lattice rows per slice chunk
  static constexpr int PPG = (kPts + NG - 1) / NG;  // points per lane group in the slice
  // LDS row stride in elements: rows of 64 bytes or more get 16 bytes of
  // padding, so lane groups reading different rows spread over the banks
  static constexpr int RS = G * (int)sizeof(TU) >= 64 ? G + 16 / (int)sizeof(TU) : G;
  // point values can be staged as whole 16-byte vectors per thread
  static constexpr bool VEC = VPT >= Vec16<TU>::N && VPT % Vec16<TU>::N == 0;
};

// LDS layout of k_splat_tile: values [P+1][G] (TU; row P stays zero) | weights [P*D] (fp32) |
// partial rows [maxq] (int32) | run starts [maxq+1] (uint16) | entry points
// [P*D] (uint8) | next unclaimed run (int32).
struct SplatLds {
  size_t w, dst, rel, lp, next, total;
};
template <typename TU>
__host__ __device__ inline SplatLds splat_lds(int P, int D, int maxq, int G) {
  SplatLds o;
  const int rs = G * (int)sizeof(TU) >= 64 ? G + 16 / (int)sizeof(TU) : G;
  size_t b = sizeof(TU) * (size_t)(P + 1) * rs;
  o.w = b;
  b += sizeof(float) * (size_t)P * D;
  o.dst = b;
  b += sizeof(int32_t) * (size_t)maxq;
  o.rel = b;
  b += sizeof(uint16_t) * (size_t)(maxq + 1);
  b = (b + 3) & ~(size_t)3;
  o.lp = b;
  b += ((size_t)P * D + 3) & ~(size_t)3;
  o.next = b;
  b += sizeof(int);
  o.total = (b + 15) & ~(size_t)15;
  return o;
}

// Scalars of k_splat_tile; its arrays are separate non-aliasing kernel
// arguments, so uniform loads (tile offsets) go through the scalar cache
// and never wait behind the tile's vector loads.
template <typename TU>
struct SplatArgs {
  int64_t n;
  int64_t items;  // tiles x channel chunks
  int P, D, C, chunks;
  int vec_v;  // V rows of a tile are one contiguous run of 16-byte vectors
  int vec_perm;  // V rows, reached through perm, are whole 16-byte vectors (C == G)
  int cvec;   // rows of C channels start 16-byte aligned
  double pp_scale;  // CG: factor of each tile's p . p (the noise variance)
  SplatLds lds;
};

// W^T restricted to one tile (Section 3.2, Splat). The block stages the
// tile's values, entries and run lists in LDS from registers that were
// loaded while the previous tile was being reduced. Each run (one lattice
// point of the tile) is summed by LPR lanes of VW channels, entries in
// order; a lane group that finishes a run claims the next unclaimed one, so
// runs of different lengths balance over the groups. The sum lands in the
// lattice point's block of partial rows (run_dst).
//
// Inside CG (up.p set, fp64) the values are the direction p in internal
// order, and the block applies the previous iteration's direction update to
// each tile as it stages it (CgDirUpdate): every (point, column) of p is
// read once here anyway, so x and p move without a pass of their own. Each
// element is read and written by the one thread that stages it; the new p
// is what the tile splats.
// DIR: the fused variant; it is launched only where a tile's values are
// all C == G columns of the direction in internal order (and whole 16-byte
// vectors, vec_v, where the shape stages vectors).
// pp (CG, else null): row t receives pp_scale * p.p of tile t per column,
// from the staged values.
template <typename TU, int G, bool DIR>
__global__ __launch_bounds__(kSplatBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_splat_tile(
    const int32_t* __restrict__ tile_off, const uint16_t* __restrict__ run_rel,
    const int32_t* __restrict__ run_dst, const uint8_t* __restrict__ ent_lp,
    const float* __restrict__ ent_w, const TU* __restrict__ V, const uint32_t* __restrict__ perm,
    TU* __restrict__ part, double* __restrict__ pp, SplatArgs<TU> a, CgDirUpdate up) {
  using S = TileShape<TU, G, kSplatBlock>;
  extern __shared__ __align__(16) unsigned char smem[];
  // CG: alpha, beta and the active flags of the columns, for the update
  __shared__ double s_alpha[DIR ? kMaxCgCols : 1], s_beta[DIR ? kMaxCgCols : 1];
  __shared__ int s_active[DIR ? kMaxCgCols : 1];
  constexpr bool upd = DIR && sizeof(TU) == 8 && S::VEC;
  TU* lv = (TU*)smem;
  float* lw = (float*)(smem + a.lds.w);
  int32_t* ldst = (int32_t*)(smem + a.lds.dst);
  uint16_t* lrel = (uint16_t*)(smem + a.lds.rel);
  uint8_t* llp = smem + a.lds.lp;
  int* lnext = (int*)(smem + a.lds.next);
  const int tid = threadIdx.x;
  constexpr int N = Vec16<TU>::N;

  TU v[S::VPT];
  float w[S::EPT];
  uint32_t lp4[S::EPT / 4];  // entry points, four per register
  uint16_t rel[S::RPT];
  int32_t dst[S::RPT];
  int nq = 0, ne = 0, q0 = 0;
  // Every load below is unconditional (indices clamped into the tile), so
  // the whole tile is in flight at once. The tile's values and entries are
  // read once per MVM: non-temporal, so that they do not push the partial
  // rows, which the gather reads next, out of the caches.
  auto fetch = [&](int64_t item) {
    const int64_t t = item / a.chunks;
    const int ch = (int)(item - t * a.chunks);
    const int64_t p0 = t * a.P;
    const int np = (int)(a.n - p0 < a.P ? a.n - p0 : a.P);
    ne = np * a.D;
    q0 = tile_off[t];
    nq = tile_off[t + 1] - q0;
    if (S::VEC && (DIR || a.vec_v)) {
      const typename Vec16<TU>::T* src = (const typename Vec16<TU>::T*)(V + p0 * a.C);
      const int nvec = np * G / N;
#pragma unroll
      for (int u = 0; u < S::VPT / N; ++u) {
        const int vi = tid + u * kSplatBlock;
        const typename Vec16<TU>::T x = __builtin_nontemporal_load(src + (vi < nvec ? vi : nvec - 1));
#pragma unroll
        for (int j = 0; j < N; ++j) v[u * N + j] = x[j];
      }
    } else if (S::VEC && a.vec_perm) {
      // rows in the caller's order: 16-byte vectors of one row each
      const int nvec = np * G / N;
#pragma unroll
      for (int u = 0; u < S::VPT / N; ++u) {
        const int vi = tid + u * kSplatBlock;
        const int f = (vi < nvec ? vi : nvec - 1) * N;
        const int64_t src = (int64_t)perm[p0 + f / G];
        const typename Vec16<TU>::T x =
            __builtin_nontemporal_load((const typename Vec16<TU>::T*)(V + src * a.C + f % G));
#pragma unroll
        for (int j = 0; j < N; ++j) v[u * N + j] = x[j];
      }
    } else {
#pragma unroll
      for (int u = 0; u < S::VPT; ++u) {
        const int f = tid + u * kSplatBlock;
        const int p = f / G < np ? f / G : np - 1;
        const int c = ch * G + f % G;
        const int64_t pt = p0 + p;
        const int64_t src = perm ? (int64_t)perm[pt] : pt;
        v[u] = V[src * a.C + (c < a.C ? c : a.C - 1)];
      }
    }
    const float* gw = ent_w + p0 * a.D;
#pragma unroll
    for (int u = 0; u < S::EPT; ++u) {
      const int e = tid + u * kSplatBlock;
      w[u] = __builtin_nontemporal_load(gw + (e < ne ? e : ne - 1));
    }
    // the tile starts 4-byte aligned (P is a multiple of 4) and the array
    // has spare bytes past its end
    const uint32_t* glp4 = (const uint32_t*)(ent_lp + p0 * a.D);
    const int nw = (ne + 3) / 4;
#pragma unroll
    for (int u = 0; u < S::EPT / 4; ++u) {
      const int wi = tid + u * kSplatBlock;
      lp4[u] = __builtin_nontemporal_load(glp4 + (wi < nw ? wi : nw - 1));
    }
#pragma unroll
    for (int u = 0; u < S::RPT; ++u) {
      const int q = tid + u * kSplatBlock;
      rel[u] = run_rel[q0 + (q < nq ? q : nq - 1)];
      dst[u] = run_dst[q0 + (q < nq ? q : nq - 1)];
    }
  };

  int64_t item, end, step;
  xcd_items(a.items, &item, &end, &step);
  for (int i = tid; i < S::RS; i += kSplatBlock) lv[a.P * S::RS + i] = (TU)0;  // the zero row
  if constexpr (upd) {
    for (int c = tid; c < a.C && c < kMaxCgCols; c += kSplatBlock) {
      s_alpha[c] = up.st->alpha[c];
      s_beta[c] = up.st->beta[c];
      s_active[c] = up.st->active[c];
    }
  }
  if (item < end) fetch(item);
  for (; item < end; item += step) {
    const int cur_nq = nq, cur_ne = ne, cur_q0 = q0;
    __syncthreads();  // the previous tile's runs are done with the LDS
    if (S::VEC && (DIR || a.vec_v || a.vec_perm)) {
      const int64_t p0 = (item / a.chunks) * a.P;
#pragma unroll
      for (int u = 0; u < S::VPT / N; ++u) {
        const int vi = tid + u * kSplatBlock;
        if (vi * N < cur_ne / a.D * G) {
          typename Vec16<TU>::T x;
          const int f = vi * N;  // N consecutive elements of one row
          if constexpr (upd) {
            // C == G here: element f of the tile is column f % G of row f / G
            typedef float fvN __attribute__((ext_vector_type(N)));
            const int64_t e = p0 * a.C + f;
            // r and x are read once here and p, x next read by other
            // kernels: streamed past the caches (non-temporal), which keeps
            // the partial rows that the gather reads next in them
            const typename Vec16<TU>::T r2 =
                __builtin_nontemporal_load((const typename Vec16<TU>::T*)((const TU*)up.r + e));
            const fvN x2 = __builtin_nontemporal_load((const fvN*)(up.x + e));
            typename Vec16<TU>::T pn;
            fvN xn;
#pragma unroll
            for (int j = 0; j < N; ++j) {
              const int c = (f + j) % G;
              const TU pold = v[u * N + j];
              xn[j] = (float)__builtin_fma(s_alpha[c], (double)pold, (double)x2[j]);
              pn[j] = s_active[c] ? (TU)__builtin_fma(s_beta[c], (double)pold, (double)r2[j]) : pold;
            }
            __builtin_nontemporal_store(pn, (typename Vec16<TU>::T*)((TU*)up.p + e));
            __builtin_nontemporal_store(xn, (fvN*)(up.x + e));
            x = pn;
          } else {
#pragma unroll
            for (int j = 0; j < N; ++j) x[j] = v[u * N + j];
          }
          *(typename Vec16<TU>::T*)(lv + (f / G) * S::RS + f % G) = x;
        }
      }
    } else {
      const int64_t p0 = (item / a.chunks) * a.P;
#pragma unroll
      for (int u = 0; u < S::VPT; ++u) {
        const int f = tid + u * kSplatBlock;
        if (f < cur_ne / a.D * G) {
          TU x = v[u];
          if constexpr (DIR && sizeof(TU) == 8 && !S::VEC) {
            // the direction update element by element (C == G here)
            const int c = f % G;
            const int64_t e = p0 * a.C + f;
            const TU pold = x;
            const double rv = __builtin_nontemporal_load((const TU*)up.r + e);
            const float xv = __builtin_nontemporal_load(up.x + e);
            x = up.st->active[c] ? (TU)__builtin_fma(up.st->beta[c], (double)pold, rv) : pold;
            __builtin_nontemporal_store(x, (TU*)up.p + e);
            __builtin_nontemporal_store((float)__builtin_fma(up.st->alpha[c], (double)pold, (double)xv), up.x + e);
          }
          lv[(f / G) * S::RS + f % G] = x;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < S::EPT; ++u) {
      const int e = tid + u * kSplatBlock;
      if (e < cur_ne) lw[e] = w[u];
    }
#pragma unroll
    for (int u = 0; u < S::EPT / 4; ++u) {
      const int wi = tid + u * kSplatBlock;
      if (4 * wi < cur_ne) ((uint32_t*)llp)[wi] = lp4[u];
    }
#pragma unroll
    for (int u = 0; u < S::RPT; ++u) {
      const int q = tid + u * kSplatBlock;
      if (q < cur_nq) {
        lrel[q] = rel[u];
        ldst[q] = dst[u];
      }
    }
    // runs past the prefetched ones (tiles with very many distinct points)
    for (int q = S::RPT * kSplatBlock + tid; q < cur_nq; q += kSplatBlock) {
      lrel[q] = run_rel[cur_q0 + q];
      ldst[q] = run_dst[cur_q0 + q];
    }
    if (tid == 0) {
      lrel[cur_nq] = (uint16_t)cur_ne;
      *lnext = S::NG;  // runs 0 .. NG-1 start on their own group
    }
    __syncthreads();
    if (item + step < end) fetch(item + step);  // in flight while this tile is reduced

    if constexpr (sizeof(TU) == 8) {
      if (pp) {
        // CG: the tile's p . p per column from the staged values, its points
        // in 16 blocks of 16, each block and then the blocks added in index
        // order, so that the sum does not depend on the channel chunk; the
        // 16 lanes of a column are consecutive (one wave)
        const int64_t tt = item / a.chunks;
        const int cc0 = (int)(item % a.chunks) * G;
        const int np = cur_ne / a.D;
        for (int pr = tid; pr < 16 * G; pr += kSplatBlock) {
          const int c = pr / 16, blk = pr % 16;
          double v = 0.0;
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int q = blk * 16 + u;
            const double x = q < np ? (double)lv[q * S::RS + c] : 0.0;
            v = __builtin_fma(x, x, v);
          }
          double tot = 0.0;
          const int l0 = (tid & 63) & ~15;
#pragma unroll
          for (int b = 0; b < 16; ++b) tot += __shfl(v, l0 + b);
          if (blk == 0 && cc0 + c < a.C) pp[tt * a.C + cc0 + c] = a.pp_scale * tot;
        }
      }
    }

    const int ch = (int)(item % a.chunks);
    const int grp = tid / S::LPR;
    const int cg = ch * G + (tid % S::LPR) * S::VW;
    const bool full = cg + S::VW <= a.C;
    int q = grp;
    if (q < cur_nq && cg < a.C) {
      int e = lrel[q], e1 = lrel[q + 1];
      int dq = ldst[q];
      TU acc[S::VW];
#pragma unroll
      for (int i = 0; i < S::VW; ++i) acc[i] = 0;
      for (;;) {
        // up to four entries of the run per pass, added in entry order
        // (a pass with fewer than four left reads the zero row with weight
        // 0 for the rest: fma(0, 0, acc) is acc exactly, as acc is never -0)
        const int cnt = e1 - e < 4 ? e1 - e : 4;
        int lpu[4];
        TU wu[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int eu = e + (u < cnt ? u : cnt - 1);
          const int lpv = (int)llp[eu];
          const float wv = lw[eu];
          lpu[u] = u < cnt ? lpv : a.P;
          wu[u] = (TU)(u < cnt ? wv : 0.f);
        }
        TU x[4][S::VW];
#pragma unroll
        for (int u = 0; u < 4; ++u) read_row<TU, S::VW>(lv + lpu[u] * S::RS + (cg - ch * G), x[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int i = 0; i < S::VW; ++i) acc[i] = fma_t(wu[u], x[u][i], acc[i]);
        e += cnt - 1;
        if (++e == e1) {
          TU* o = part + (int64_t)dq * a.C + cg;
          if (full && a.cvec) {
            write_row<TU, S::VW>(o, acc);
          } else {
#pragma unroll
            for (int i = 0; i < S::VW; ++i)
              if (cg + i < a.C) o[i] = acc[i];
          }
          // next run: whichever is unclaimed (one group's lanes share it);
          // a run's sum does not depend on which group takes it
          int nx = 0;
          if (tid % S::LPR == 0) nx = atomicAdd(lnext, 1);
          q = __shfl(nx, tid - tid % S::LPR);
          if (q >= cur_nq) break;
          e = lrel[q];
          e1 = lrel[q + 1];
          dq = ldst[q];
#pragma unroll
          for (int i = 0; i < S::VW; ++i) acc[i] = 0;
        }
      }
    }
  }
}

// U[j] = sum of lattice point j's partial rows occ_ptr[j] .. occ_ptr[j+1]-1
// (one per piece of a run touching it, contiguous; row_vert names each row's
// lattice point). The rows are cut into ranges of R rows (gather_rows); a
// group of G lanes adds its range's rows in order, eight rows loaded at a
// time.
// A lattice point whose rows lie in one range is written directly; the part
// of a longer one that a range holds becomes a fragment (slot 0: it starts
// the range; slot 1: it ends the range), summed in range order by
// k_gather_fix. The work per group is fixed, whatever the list lengths.
// VW channels per lane (16-byte loads when the rows allow), G / VW lanes per
// group; every channel's rows are added in the same order for any VW.
template <typename TU, int G, int VW>
__global__ __launch_bounds__(kBlock) void k_splat_gather(const int32_t* __restrict__ row_vert,
                                                         const TU* __restrict__ part,
                                                         TU* __restrict__ U, TU* __restrict__ frag,
                                                         int64_t nrows, int C, int64_t ngroups, int R) {
  constexpr int LG = G / VW;       // lanes per group
  constexpr int GPB = kBlock / LG;  // groups per block
  constexpr int B = 8;              // rows loaded together
  const int lane = threadIdx.x % LG;
  const int64_t gi = xcd_block(blockIdx.x, gridDim.x) * GPB + threadIdx.x / LG;
  if (gi >= ngroups) return;
  const int64_t o0 = gi * R;
  const int64_t o1 = o0 + R < nrows ? o0 + R : nrows;
  // a segment is a whole lattice point unless it touches a range edge that
  // its lattice point continues across
  const int32_t before = o0 > 0 ? row_vert[o0 - 1] : -1;
  const int32_t after = o1 < nrows ? row_vert[o1] : -1;
  for (int c = lane * VW; c < C; c += G) {
    int32_t cur = row_vert[o0];
    int64_t seg = o0;
    TU acc[VW];
#pragma unroll
    for (int i = 0; i < VW; ++i) acc[i] = 0;
    auto flush = [&](int64_t end) {
      const bool whole = (seg > o0 || before != cur) && (end < o1 || after != cur);
      TU* dst = whole ? U + (int64_t)cur * C + c : frag + (gi * 2 + (seg == o0 ? 0 : 1)) * C + c;
      write_row<TU, VW>(dst, acc);
    };
    for (int64_t k0 = o0; k0 < o1; k0 += B) {
      TU v[B][VW];
      int32_t rv[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int64_t k = k0 + u < o1 ? k0 + u : o1 - 1;
        // partial rows are read once: non-temporal, which keeps the
        // lattice values the blur reads next in the caches
        read_row_nt<TU, VW>(part + k * C + c, v[u]);
        rv[u] = row_vert[k];
      }
#pragma unroll
      for (int u = 0; u < B; ++u) {
        if (k0 + u < o1) {
          if (rv[u] != cur) {
            flush(k0 + u);
            cur = rv[u];
            seg = k0 + u;
#pragma unroll
            for (int i = 0; i < VW; ++i) acc[i] = 0;
          }
#pragma unroll
          for (int i = 0; i < VW; ++i) acc[i] += v[u][i];
        }
      }
    }
    flush(o1);
  }
}

// Lattice points whose rows span several ranges: each is summed from its
// fragments in range order by the range its rows end in (one thread per
// (range, channel); a range's first row belongs to the lattice point that
// may continue into it).
__global__ __launch_bounds__(kBlock) void k_gather_fix(const int32_t* __restrict__ row_vert,
                                                       const int32_t* __restrict__ occ_ptr,
                                                       const void* __restrict__ frag_v,
                                                       void* __restrict__ U_v, int64_t ngroups, int C,
                                                       int elem, int R) {
  const int64_t total = ngroups * C;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += stride) {
    const int64_t g1 = q / C;
    const int c = (int)(q - g1 * C);
    if (g1 == 0) continue;
    const int64_t j = row_vert[g1 * R];
    const int64_t js = occ_ptr[j], je = occ_ptr[j + 1];
    const int64_t g0 = js / R;
    if (g0 == g1 || (je - 1) / R != g1) continue;  // starts here, or ends further on
    const int64_t first = (g0 * 2 + (js == g0 * R ? 0 : 1)) * C + c;
    if (elem == 8) {
      const double* frag = (const double*)frag_v;
      double acc = frag[first];
      for (int64_t g = g0 + 1; g <= g1; ++g) acc += frag[(g * 2) * C + c];
      ((double*)U_v)[j * C + c] = acc;
    } else {
      const float* frag = (const float*)frag_v;
      float acc = frag[first];
      for (int64_t g = g0 + 1; g <= g1; ++g) acc += frag[(g * 2) * C + c];
      ((float*)U_v)[j * C + c] = acc;
    }
  }
}

template <typename TU>
struct BlurArgs {
  const TU* in[2];
  TU* out[2];
  const int32_t* nbr[2];  // this step's direction per chain: [point][offset], 2r per point
  int64_t m;
  int C;
  int r;
  int chains;
  int sum_out;  // last SYMMETRIC step: out[0] = forward + reverse
  int vec;      // rows of C channels start 16-byte aligned
  int nt;       // lattice values exceed the Infinity Cache: stream the outputs past it
  int64_t rows_per_block;
  TU st[2 * kMaxOrder + 1];
};

// One chain's blur of VW channels of row j: sum over t = -r..r of
// stencil[t] * U[neighbour(j, t)], in t order; a missing neighbour adds 0.
template <typename TU, int VW>
__device__ __forceinline__ void load_vw(const TU* __restrict__ in, int64_t row, int64_t valid, int C, int c,
                                        bool vec, TU (&v)[VW]);

template <typename TU, int VW>
__device__ __forceinline__ void blur_rows(const TU* __restrict__ in, const int32_t* __restrict__ nb,
                                          int64_t j, int C, int c, int r, const TU* st, bool vec,
                                          TU (&acc)[VW]) {
#pragma unroll
  for (int i = 0; i < VW; ++i) acc[i] = 0;
  if (r == 1) {
    // the three-tap stencil: both neighbour indices (one 8-byte load), then
    // the three rows, in flight together
    const int2 lh = *(const int2*)(nb + 2 * j);
    const int64_t lo = lh.x, hi = lh.y;
    TU v[3][VW];
    load_vw<TU, VW>(in, lo, j, C, c, vec, v[0]);
    load_vw<TU, VW>(in, j, j, C, c, vec, v[1]);
    load_vw<TU, VW>(in, hi, j, C, c, vec, v[2]);
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
      for (int i = 0; i < VW; ++i) acc[i] = fma_t(st[t], v[t][i], acc[i]);
    return;
  }
  // neighbour rows first (2r independent loads), then the values
  int32_t nbv[2 * kMaxOrder];
  for (int ti = 0; ti < 2 * r; ++ti) nbv[ti] = nb[j * (2 * r) + ti];
  int ti = 0;
  for (int t = -r; t <= r; ++t) {
    const int64_t row = t == 0 ? j : (int64_t)nbv[ti++];
    TU v[VW];
    load_vw<TU, VW>(in, row, j, C, c, vec, v);
#pragma unroll
    for (int i = 0; i < VW; ++i) acc[i] = fma_t(st[t + r], v[i], acc[i]);
  }
}

template <int G>
__host__ __device__ constexpr int blur_vw() { return G < 4 ? G : 4; }

// One thread per (row, VW channels).
template <typename TU, int G>
__global__ __launch_bounds__(kBlock) void k_blur(BlurArgs<TU> a) {
  constexpr int VW = blur_vw<G>();
  constexpr int LPR = G / VW;
  constexpr int R = kBlock / LPR;
  const int sub = threadIdx.x % LPR;
  const int64_t j0 = xcd_block(blockIdx.x, gridDim.x) * a.rows_per_block;
  const int64_t j1 = j0 + a.rows_per_block < a.m ? j0 + a.rows_per_block : a.m;
  for (int64_t j = j0 + threadIdx.x / LPR; j < j1; j += R) {
    for (int c = sub * VW; c < a.C; c += G) {
      const bool vec = a.vec && c + VW <= a.C;
      TU f[VW];
      blur_rows<TU, VW>(a.in[0], a.nbr[0], j, a.C, c, a.r, a.st, vec, f);
      if (a.chains == 2) {
        TU b[VW];
        blur_rows<TU, VW>(a.in[1], a.nbr[1], j, a.C, c, a.r, a.st, vec, b);
        if (a.sum_out) {
#pragma unroll
          for (int i = 0; i < VW; ++i) f[i] = f[i] + b[i];
        } else {
          TU* o1 = a.out[1] + j * a.C + c;
          if (vec) {
            if (a.nt)
              write_row_nt<TU, VW>(o1, b);
            else
              write_row<TU, VW>(o1, b);
          } else {
#pragma unroll
            for (int i = 0; i < VW; ++i)
              if (c + i < a.C) o1[i] = b[i];
          }
        }
      }
      TU* o0 = a.out[0] + j * a.C + c;
      if (vec) {
        if (a.nt)
          write_row_nt<TU, VW>(o0, f);
        else
          write_row<TU, VW>(o0, f);
      } else {
#pragma unroll
        for (int i = 0; i < VW; ++i)
          if (c + i < a.C) o0[i] = f[i];
      }
    }
  }
}

// Two consecutive blur steps in one launch, for a 3-tap stencil (r = 1):
// out(j) = sum over t2 of st[t2] * B(neighbour2(j, t2)), where B(x) = sum
// over t1 of st[t1] * in(neighbour1(x, t1)) is the first step's value at x,
// formed here in the same order as a launch of its own would form it (a
// missing lattice point contributes 0). Nine rows per output row instead of
// two launches of three; the rows mostly come from L2 and MALL.
template <typename TU>
struct Blur2Args {
  const TU* in[2];
  TU* out[2];
  const int32_t* nbr1[2];  // first step's direction, per chain ([point][offset])
  const int32_t* nbr2[2];  // second step's direction
  int64_t m;
  int C;
  int chains;
  int sum_out;
  int split;  // two chains with outputs of their own: the grid's halves take one each
  int chain0; // k_blur2_split: the first half's chain
  int halves; // k_blur2_split: 2 (both chains) or 1 (chain0 alone)
  int vec;
  int nt;     // as in BlurArgs
  int64_t rows_per_block;
  TU st[3];
};

// VW values of a lattice row, or zeros where row < 0 (a missing neighbour).
// The load is issued unconditionally (from row `valid` when row < 0) and the
// zeros selected afterwards, so a thread's loads never wait on one another
// through a branch.
template <typename TU, int VW>
__device__ __forceinline__ void load_vw(const TU* __restrict__ in, int64_t row, int64_t valid, int C, int c,
                                        bool vec, TU (&v)[VW]) {
  const TU* src = in + (row >= 0 ? row : valid) * C + c;
  if (vec) {
    read_row<TU, VW>(src, v);
  } else {
#pragma unroll
    for (int i = 0; i < VW; ++i) {
      const TU x = src[c + i < C ? i : 0];
      v[i] = c + i < C ? x : (TU)0;
    }
  }
#pragma unroll
  for (int i = 0; i < VW; ++i) v[i] = row >= 0 ? v[i] : (TU)0;
}

template <typename TU, int VW>
__device__ __forceinline__ void blur2_rows(const TU* __restrict__ in, const int32_t* __restrict__ nb1,
                                           const int32_t* __restrict__ nb2, int64_t j, int C, int c,
                                           const TU* st, bool vec, TU (&acc)[VW]) {
  // second-direction neighbours of j (t2 = -1, 0, +1), then their
  // first-direction neighbours, then the nine rows
  int64_t x[3];
  const int2 lh2 = *(const int2*)(nb2 + 2 * j);
  x[0] = lh2.x;
  x[1] = j;
  x[2] = lh2.y;
  // (all six index loads and all nine row loads issue without waiting on
  // one another: indices of a missing x are read at j and discarded)
  int64_t y[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int64_t xa = x[a] >= 0 ? x[a] : j;
    const int2 lh1 = *(const int2*)(nb1 + 2 * xa);
    y[a][0] = x[a] >= 0 ? (int64_t)lh1.x : -1;
    y[a][1] = x[a];
    y[a][2] = x[a] >= 0 ? (int64_t)lh1.y : -1;
  }
  TU v[3][3][VW];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) load_vw<TU, VW>(in, y[a][b], j, C, c, vec, v[a][b]);
#pragma unroll
  for (int i = 0; i < VW; ++i) acc[i] = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    TU bx[VW];
#pragma unroll
    for (int i = 0; i < VW; ++i) bx[i] = 0;
    if (x[a] >= 0) {
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int i = 0; i < VW; ++i) bx[i] = fma_t(st[b], v[a][b][i], bx[i]);
    }
#pragma unroll
    for (int i = 0; i < VW; ++i) acc[i] = fma_t(st[a], bx[i], acc[i]);
  }
}

template <typename TU, int G>
__global__ __launch_bounds__(kBlock) void k_blur2(Blur2Args<TU> a) {
  constexpr int VW = blur_vw<G>();
  constexpr int LPR = G / VW;
  constexpr int R = kBlock / LPR;
  const int sub = threadIdx.x % LPR;
  const int64_t j0 = xcd_block(blockIdx.x, gridDim.x) * a.rows_per_block;
  const int64_t j1 = j0 + a.rows_per_block < a.m ? j0 + a.rows_per_block : a.m;
  for (int64_t j = j0 + threadIdx.x / LPR; j < j1; j += R) {
    for (int c = sub * VW; c < a.C; c += G) {
      const bool vec = a.vec && c + VW <= a.C;
      TU f[VW];
      blur2_rows<TU, VW>(a.in[0], a.nbr1[0], a.nbr2[0], j, a.C, c, a.st, vec, f);
      if (a.chains == 2) {
        TU b[VW];
        blur2_rows<TU, VW>(a.in[1], a.nbr1[1], a.nbr2[1], j, a.C, c, a.st, vec, b);
        if (a.sum_out) {
#pragma unroll
          for (int i = 0; i < VW; ++i) f[i] = f[i] + b[i];
        } else {
          TU* o1 = a.out[1] + j * a.C + c;
          if (vec) {
            if (a.nt)
              write_row_nt<TU, VW>(o1, b);
            else
              write_row<TU, VW>(o1, b);
          } else {
#pragma unroll
            for (int i = 0; i < VW; ++i)
              if (c + i < a.C) o1[i] = b[i];
          }
        }
      }
      TU* o0 = a.out[0] + j * a.C + c;
      if (vec) {
        if (a.nt)
          write_row_nt<TU, VW>(o0, f);
        else
          write_row<TU, VW>(o0, f);
      } else {
#pragma unroll
        for (int i = 0; i < VW; ++i)
          if (c + i < a.C) o0[i] = f[i];
      }
    }
  }
}

// k_blur2 for two chains that write outputs of their own: the grid's first
// half takes chain 0 and its second half chain 1, the same rows each, so a
// thread waits on half as many dependent loads.
template <typename TU, int G>
__global__ __launch_bounds__(kBlock) void k_blur2_split(Blur2Args<TU> a) {
  constexpr int VW = blur_vw<G>();
  constexpr int LPR = G / VW;
  constexpr int R = kBlock / LPR;
  const int sub = threadIdx.x % LPR;
  const unsigned nb = gridDim.x / a.halves;
  const int half = blockIdx.x >= nb ? 1 : 0;
  const int chain = a.chain0 + half;
  const unsigned bid = blockIdx.x - half * nb;
  const int64_t j0 = xcd_block(bid, nb) * a.rows_per_block;
  const int64_t j1 = j0 + a.rows_per_block < a.m ? j0 + a.rows_per_block : a.m;
  for (int64_t j = j0 + threadIdx.x / LPR; j < j1; j += R) {
    for (int c = sub * VW; c < a.C; c += G) {
      const bool vec = a.vec && c + VW <= a.C;
      TU f[VW];
      blur2_rows<TU, VW>(a.in[chain], a.nbr1[chain], a.nbr2[chain], j, a.C, c, a.st, vec, f);
      TU* o = a.out[chain] + j * a.C + c;
      if (vec) {
        if (a.nt)
          write_row_nt<TU, VW>(o, f);
        else
          write_row<TU, VW>(o, f);
      } else {
#pragma unroll
        for (int i = 0; i < VW; ++i)
          if (c + i < a.C) o[i] = f[i];
      }
    }
  }
}

// LDS layout of k_slice_tile: lattice rows [RC][G] (TU; also the CG
// reduction area) | weights [P*D] (fp32) | slots [P*D] (uint16).
struct SliceLds {
  size_t w, sl, total;
  int zrow;  // an all-zero lattice row past the staged rows and the reduction area
};
template <typename TU, int G, int NT = 1024>
__host__ __device__ inline SliceLds slice_lds(int P, int D, int maxq) {
  using S = TileShape<TU, G, NT>;
  SliceLds o;
  const size_t row = sizeof(TU) * (size_t)S::RS;
  size_t b = row * (size_t)S::RC;
  const size_t red = sizeof(double) * (256 * 16 + 16 * 16);  // CG tile reduction
  if (b < red) b = red;
  o.zrow = (int)((b + row - 1) / row);
  b = row * (size_t)(o.zrow + 1);
  o.w = b;
  b += sizeof(float) * (size_t)P * D;
  o.sl = b;
  b += sizeof(uint16_t) * (size_t)(P * D + 1);
  o.total = (b + 15) & ~(size_t)15;
  return o;
}

// Scalars of k_slice_tile (its arrays are separate non-aliasing kernel
// arguments, as in k_splat_tile).
template <typename TU>
struct SliceArgs {
  int64_t n;
  int64_t items;
  int P, D, C, chunks;
  int cvec;
  TU scale;
  TU noise;
  int64_t mrows;        // CG: rows whose caller index is >= mrows are not solved for
  SliceLds lds;
};

// out = scale * W U restricted to one tile (Section 3.2, Slice). The tile's
// (slot, weight) entries and its first RC lattice rows arrive in registers
// while the previous tile is computed; a tile with more runs stages the rest
// RC rows at a time. Each point is combined by LPR lanes of VW channels from
// the staged rows. The CG variant forms q = out + noise * p, moves the
// residual (out is r: r -= alpha q, alpha already known) and emits the
// tile's new r . r per column, reduced in a fixed order.
template <typename TU, int G, bool CG, int NT>
// perm: caller row of each sorted point, or null. CG only: p is the
// direction and out the residual (sorted order), hook.partials receive each
// tile's r . r per column, mperm maps sorted points to caller rows for the
// mrows mask.
__global__ __launch_bounds__(NT) void k_slice_tile(
    const int32_t* __restrict__ tile_off, const int32_t* __restrict__ tile_verts,
    const uint16_t* __restrict__ loc, const float* __restrict__ ws, const TU* __restrict__ U,
    TU* __restrict__ out, const uint32_t* __restrict__ perm, const TU* __restrict__ p,
    CgHook hook, const uint32_t* __restrict__ mperm, SliceArgs<TU> a) {
  using S = TileShape<TU, G, NT>;
  static_assert(S::RC % kSliceOrderRows == 0, "staged chunks hold whole order blocks");
  extern __shared__ __align__(16) unsigned char smem[];
  TU* lu = (TU*)smem;
  float* lw = (float*)(smem + a.lds.w);
  uint16_t* lsl = (uint16_t*)(smem + a.lds.sl);
  const int tid = threadIdx.x;
  constexpr int RC = S::RC;

  float w[S::EPT];
  uint32_t sl2[S::EPT / 2];  // two 16-bit slots per register
  TU ur[S::UPT];
  int nq = 0, np = 0, q0 = 0;
  // rows [r0, r0 + nr) (nr >= 1) of a tile's run list, whose lattice points
  // are verts[r0 ..]. Indices past the end are clamped to valid ones, so all
  // index loads issue before the row loads that depend on them.
  int32_t vj[S::UPT];
  auto load_index = [&](int r0, int nr, const int32_t* verts) {
#pragma unroll
    for (int u = 0; u < S::UPT; ++u) {
      const int r = (tid + u * S::NT) / G;
      vj[u] = verts[r0 + (r < nr ? r : nr - 1)];
    }
  };
  auto load_rows = [&](int ch) {
#pragma unroll
    for (int u = 0; u < S::UPT; ++u) {
      const int c = ch * G + (tid + u * S::NT) % G;
      ur[u] = U[(int64_t)vj[u] * a.C + (c < a.C ? c : a.C - 1)];
    }
  };
  // A tile's first-chunk row indices are requested early (fetch_index) and
  // its entries and rows later (fetch), so the rows never wait for them.
  auto fetch_index = [&](int64_t item) {
    const int64_t t = item / a.chunks;
    const int64_t p0 = t * a.P;
    np = (int)(a.n - p0 < a.P ? a.n - p0 : a.P);
    q0 = tile_off[t];
    nq = tile_off[t + 1] - q0;
    load_index(0, nq < RC ? nq : RC, tile_verts + q0);
  };
  auto fetch = [&](int64_t item) {
    const int64_t t = item / a.chunks;
    const int ch = (int)(item - t * a.chunks);
    const int64_t p0 = t * a.P;
    const int ne = np * a.D;
    const float* gw = ws + p0 * a.D;
    const uint16_t* gsl = loc + p0 * a.D;
#pragma unroll
    for (int u = 0; u < S::EPT; ++u) {
      const int e = tid + u * S::NT;
      w[u] = gw[e < ne ? e : ne - 1];
    }
    // slots in pairs (the tile starts 4-byte aligned; the array has a
    // spare slot past its end)
    const uint32_t* gsl2 = (const uint32_t*)gsl;
    const int npair = (ne + 1) / 2;
#pragma unroll
    for (int u = 0; u < S::EPT / 2; ++u) {
      const int pi = tid + u * S::NT;
      sl2[u] = gsl2[pi < npair ? pi : npair - 1];
    }
    load_rows(ch);
  };
  auto stage_rows = [&](int nr) {
#pragma unroll
    for (int u = 0; u < S::UPT; ++u) {
      const int f = tid + u * S::NT;
      if (f < nr * G) lu[(f / G) * S::RS + f % G] = ur[u];
    }
  };

  // CG: alpha of every column (known before this kernel)
  __shared__ TU s_alpha[CG ? kMaxCgCols : 1];
  if constexpr (CG) {
    for (int c = tid; c < a.C && c < kMaxCgCols; c += S::NT) s_alpha[c] = (TU)hook.st->alpha[c];
  }
  int64_t item, end, step;
  xcd_items(a.items, &item, &end, &step);
  for (int i = tid; i < S::RS; i += S::NT) lu[a.lds.zrow * S::RS + i] = (TU)0;  // the zero row
  if (item < end) {
    fetch_index(item);
    fetch(item);
  }
  for (; item < end; item += step) {
    const int64_t t = item / a.chunks;
    const int ch = (int)(item - t * a.chunks);
    const int cur_nq = nq, cur_np = np, cur_ne = np * a.D, cur_q0 = q0;
    __syncthreads();  // the previous tile is done with the LDS
#pragma unroll
    for (int u = 0; u < S::EPT; ++u) {
      const int e = tid + u * S::NT;
      if (e < cur_ne) lw[e] = w[u];
    }
#pragma unroll
    for (int u = 0; u < S::EPT / 2; ++u) {
      const int pi = tid + u * S::NT;
      if (2 * pi < cur_ne) ((uint32_t*)lsl)[pi] = sl2[u];
    }
    stage_rows(cur_nq < RC ? cur_nq : RC);

    const int grp = tid / S::LPR;
    const int cl = (tid % S::LPR) * S::VW;  // channel offset within the chunk
    const int cg = ch * G + cl;
    const bool live = cg < a.C;
    const bool full = cg + S::VW <= a.C;
    // CG: this thread's p and r values, requested before the next tile's
    // loads so that using them never waits for those
    TU pv[S::PPG][S::VW], rv[S::PPG][S::VW];
#pragma unroll
    for (int k = 0; k < S::PPG; ++k) {
      const int lp = grp + k * S::NG;
#pragma unroll
      for (int i = 0; i < S::VW; ++i) {
        pv[k][i] = 0;
        rv[k][i] = 0;
      }
      if (CG && lp < cur_np && live) {
        const int64_t pt = t * a.P + lp;
        const TU* src = p + pt * a.C + cg;
        const TU* rsrc = out + pt * a.C + cg;
        if (full && a.cvec) {
          read_row<TU, S::VW>(src, pv[k]);
          read_row<TU, S::VW>(rsrc, rv[k]);
        } else {
#pragma unroll
          for (int i = 0; i < S::VW; ++i)
            if (cg + i < a.C) {
              pv[k][i] = src[i];
              rv[k][i] = rsrc[i];
            }
        }
      }
    }

    const bool next = item + step < end;
    if (next) fetch_index(item + step);
    TU acc[S::PPG][S::VW];
#pragma unroll
    for (int k = 0; k < S::PPG; ++k)
#pragma unroll
      for (int i = 0; i < S::VW; ++i) acc[k][i] = 0;
    for (int r0 = 0; r0 < cur_nq; r0 += RC) {
      const int nr = cur_nq - r0 < RC ? cur_nq - r0 : RC;
      if (r0 > 0) {
        __syncthreads();  // previous chunk consumed
        load_index(r0, nr, tile_verts + cur_q0);
        load_rows(ch);
        stage_rows(nr);
        if (next) fetch_index(item + step);  // the indices were overwritten
      }
      __syncthreads();
      // the next tile's entries and first rows load during the last chunk
      if (r0 + RC >= cur_nq && next) fetch(item + step);
      if (live) {
#pragma unroll
        for (int k = 0; k < S::PPG; ++k) {
          const int lp = grp + k * S::NG;
          if (lp < cur_np) {
            const int eb = lp * a.D;
            // EB entries at a time: slots and weights, then their rows
            constexpr int EB = S::VW * sizeof(TU) >= 32 ? (CG ? 1 : 2) : 4;
            // A point's entries are added by block of kSliceOrderRows runs
            // of the tile's run list, then in vertex order, whatever RC is
            // (a multiple of that block): the sums do not depend on the
            // channel chunk or block shape.
            // An entry outside the block (or past the point's d+1) reads
            // the zero row with weight 0: fma(0, 0, acc) is acc exactly, as
            // acc is never -0.
            for (int s0 = 0; s0 < nr; s0 += kSliceOrderRows)
            for (int j0 = 0; j0 < a.D; j0 += EB) {
              int sv[EB];
              TU wv[EB];
#pragma unroll
              for (int u = 0; u < EB; ++u) {
                const int j = j0 + u < a.D ? j0 + u : a.D - 1;
                const int sr = (int)lsl[eb + j] - r0 - s0;
                const float wr = lw[eb + j];
                const bool in = (unsigned)sr < (unsigned)(nr - s0 < kSliceOrderRows ? nr - s0 : kSliceOrderRows) &&
                                j0 + u < a.D;
                sv[u] = in ? s0 + sr : a.lds.zrow;
                wv[u] = (TU)(in ? wr : 0.f);
              }
              TU x[EB][S::VW];
#pragma unroll
              for (int u = 0; u < EB; ++u) read_row<TU, S::VW>(lu + sv[u] * S::RS + cl, x[u]);
#pragma unroll
              for (int u = 0; u < EB; ++u)
#pragma unroll
                for (int i = 0; i < S::VW; ++i) acc[k][i] = fma_t(wv[u], x[u][i], acc[k][i]);
            }
          }
        }
      }
    }
    double prod[S::PPG][S::VW];  // CG: r . r of each (point, channel)
#pragma unroll
    for (int k = 0; k < S::PPG; ++k) {
      const int lp = grp + k * S::NG;
#pragma unroll
      for (int i = 0; i < S::VW; ++i) prod[k][i] = 0.0;
      if (lp < cur_np && live) {
        const int64_t pt = t * a.P + lp;
        TU o[S::VW];
        const bool masked = CG && a.mrows > 0 && (int64_t)mperm[pt] >= a.mrows;  // not solved for
#pragma unroll
        for (int i = 0; i < S::VW; ++i) {
          o[i] = a.scale * acc[k][i];
          if (CG) {
            const TU q = masked ? (TU)0 : fma_t(a.noise, pv[k][i], o[i]);
            o[i] = fma_t(-s_alpha[cg + i < a.C ? cg + i : 0], q, rv[k][i]);
            prod[k][i] = (double)o[i] * (double)o[i];
          }
        }
        TU* dstp = out + (perm ? (int64_t)perm[pt] : pt) * a.C + cg;
        if (full && a.cvec) {
          write_row<TU, S::VW>(dstp, o);
        } else {
#pragma unroll
          for (int i = 0; i < S::VW; ++i)
            if (cg + i < a.C) dstp[i] = o[i];
        }
      }
    }
    if (CG) {
      // the tile's r . r per column: points in 16 blocks of 16, each block
      // and then the blocks added in index order, so that the sum does not
      // depend on how channels are split over lanes; 16 channels per pass
      double* sh = (double*)smem;            // [256 points][16 channels]
      double* sh2 = sh + 256 * 16;           // [16 blocks][16 channels]
      for (int cs = 0; cs < G; cs += 16) {
        __syncthreads();  // every lane is done with the staged rows / last pass
#pragma unroll
        for (int k = 0; k < S::PPG; ++k) {
          const int lp = grp + k * S::NG;
#pragma unroll
          for (int i = 0; i < S::VW; ++i) {
            const int cc = cl + i - cs;
            if (lp < 256 && cc >= 0 && cc < 16) sh[lp * 16 + cc] = prod[k][i];
          }
        }
        __syncthreads();
        if (tid < 256) {
          // every row is read (rows past the tile hold stale values and add
          // nothing), so the reads need no branches
          const int c16 = tid % 16, blk = tid / 16;
          const double* src = sh + blk * 256 + c16;
          double x[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) x[u] = src[u * 16];
          double v = 0.0;
#pragma unroll
          for (int u = 0; u < 16; ++u) v += blk * 16 + u < cur_np ? x[u] : 0.0;
          sh2[blk * 16 + c16] = v;
        }
        __syncthreads();
        if (tid < 16 && cs + tid < G && ch * G + cs + tid < a.C) {
          double v = 0.0;
          for (int blk = 0; blk < 16; ++blk) v += sh2[blk * 16 + tid];
          hook.partials[t * a.C + ch * G + cs + tid] = v;
        }
      }
    }
  }
  // CG: the last block to finish folds the tiles' r . r into beta
  if constexpr (CG) cg_finish(hook, a.C, (double*)smem);
}


template <typename TU>
size_t slice_lds_g(int P, int D, int maxq, int g) {
  switch (g) {
    case 1: return slice_lds<TU, 1>(P, D, maxq).total;
    case 2: return slice_lds<TU, 2>(P, D, maxq).total;
    case 4: return slice_lds<TU, 4>(P, D, maxq).total;
    case 8: return slice_lds<TU, 8>(P, D, maxq).total;
    default: return slice_lds<TU, 16>(P, D, maxq).total;
  }
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

int cu_count() {
  constexpr int kMaxDevices = 64;
  static int cus[kMaxDevices] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 256;
  if (!cus[dev]) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1) c = 256;
    cus[dev] = c;
  }
  return cus[dev];
}

// Blocks of a persistent tile kernel: as many as can be resident, at most
// one per work item. A kernel staging more than 64 KiB of LDS is first
// allowed to.
// Launch choices an autotuning run can set: the channel chunk width and the
// resident blocks per CU of the persistent splat and slice (0: as many as
// the occupancy allows). None of them changes a result: every sum is formed
// in an order that depends on neither the chunk width nor the grid.
struct LaunchChoice {
  int g;
  int splat_bpc;
  int slice_bpc;
};
struct TuneEntry {
  int d, elem, g0, mlog;
  LaunchChoice c;
  float ms;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;                  // process-wide, keyed by lattice shape
thread_local const LaunchChoice* g_force = nullptr;  // set while candidates are timed

int mlog_of(int64_t m) {
  int b = 0;
  while (((int64_t)1 << b) < m) ++b;
  return b;
}

bool tune_find(const sgp_lattice* L, int C, int elem, LaunchChoice* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const TuneEntry& e : g_tune)
    if (e.d == L->d && e.elem == elem && e.g0 == lanes_for(C) && e.mlog == mlog_of(L->m)) {
      *out = e.c;
      return true;
    }
  return false;
}

unsigned persistent_grid(const void* kernel, int threads, size_t lds, int64_t items, int chosen_bpc) {
  if (lds > 65536) (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  (void)hipGetLastError();
  int bpc = tuning().blocks_per_cu;
  if (bpc <= 0) bpc = chosen_bpc;
  if (bpc <= 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, lds) != hipSuccess || nb < 1) {
      (void)hipGetLastError();
      nb = 1;
    }
    bpc = nb;
  }
  int64_t g = (int64_t)cu_count() * bpc;
  if (g > items) g = items;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// Rows per gather range: 64, halved (down to 8) while the lattice would
// have fewer than 4096 ranges, so that a small lattice's gather still
// spreads over the GPU instead of summing long ranges in few groups.
int gather_rows(const sgp_lattice* L) {
  int r = 64;
  while (r > 8 && (L->npiece + r - 1) / r < 4096) r >>= 1;
  return r;
}
int64_t gather_ranges(const sgp_lattice* L) {
  const int r = gather_rows(L);
  return (L->npiece + r - 1) / r;
}

unsigned grid_cap(int64_t work) {
  int64_t b = (work + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return (unsigned)b;
}

// Blocks for `rows` rows at R per block, capped, and the rows each block
// takes so that the blocks cover all rows.
void split_rows(int64_t rows, int R, int64_t cap, unsigned* blocks, int64_t* rows_per_block) {
  int64_t b = (rows + R - 1) / R;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  *rows_per_block = (rows + b - 1) / b;
  *blocks = (unsigned)((rows + *rows_per_block - 1) / *rows_per_block);
}

// Work memory of one MVM in elements of its accumulator type: four m x C
// lattice value arrays (the splat's result and the blur's ping-pong; a
// fifth inside CG, where the splat's result must outlive the blur), one
// partial row per run piece, two fragment rows per gather range.
size_t mvm_work_elems(const sgp_lattice* L, int C, bool cg) {
  return (size_t)((cg ? 5 : 4) * L->m + L->npiece + 2 * gather_ranges(L)) * (size_t)C;
}

// cgm (CG only, else null): V is the direction p, out the residual r (both
// internal order), and the MVM finishes the CG step (CgMvm).
template <typename TU, int G>
int mvm_g(const sgp_lattice* L, const TU* V, const uint32_t* perm, int C, TU* out, hipStream_t s,
          TU noise, const CgMvm* cgm, const LaunchChoice& lc, void* work, const CgDirUpdate* up) {
  const int d = L->d, D = d + 1, T = 2 * L->order;
  const int64_t m = L->m, mC = m * C;
  const TU* p = cgm ? V : nullptr;
  TU* U0 = (TU*)work;
  TU* B1 = U0 + mC;
  TU* B2 = B1 + mC;
  TU* B3 = B2 + mC;
  TU* B4 = cgm ? B3 + mC : U0;  // chain 1's second array (U0 itself outside CG)
  TU* part = (cgm ? B4 : B3) + mC;
  TU* frag = part + L->npiece * C;  // 2 rows per gather range
  const int chunks = (C + G - 1) / G;
  const int P = L->tile_points;
  const dim3 tgrid((unsigned)L->ntiles, (unsigned)chunks);
  const int maxq = L->max_tile_runs;
  SplatArgs<TU> sa;
  sa.n = L->n;
  sa.items = L->ntiles * chunks;
  sa.P = P;
  sa.D = D;
  sa.C = C;
  sa.chunks = chunks;
  sa.vec_v = (TileShape<TU, G, kSplatBlock>::VEC && !perm && C == G && aligned16(V)) ? 1 : 0;
  sa.vec_perm = (TileShape<TU, G, kSplatBlock>::VEC && perm && C == G && aligned16(V)) ? 1 : 0;
  sa.cvec = (C % Vec16<TU>::N == 0 && aligned16(part)) ? 1 : 0;
  sa.lds = splat_lds<TU>(P, D, L->max_tile_pieces, G);
  sa.pp_scale = cgm ? (double)noise : 0.0;
  double* pp = cgm ? cgm->pp : nullptr;
  // the previous CG iteration's direction update: in this splat where its
  // values are whole vectors of all C columns, else as a pass of its own
  const bool dir_fused = up && sizeof(TU) == 8 && !perm && C == G &&
                         (!TileShape<TU, G, kSplatBlock>::VEC || sa.vec_v);
  if (up && !dir_fused) {
    const int rc = launch_cg_dir(*up, (int64_t)L->n * C, C, s);
    if (rc) return rc;
  }
  {
    ProfScope ps(KK_SPLAT, s);
    const void* kern =
        dir_fused ? (const void*)&k_splat_tile<TU, G, true> : (const void*)&k_splat_tile<TU, G, false>;
    const unsigned grid = persistent_grid(kern, kSplatBlock, sa.lds.total, sa.items, lc.splat_bpc);
    if (dir_fused)
      hipLaunchKernelGGL((k_splat_tile<TU, G, true>), dim3(grid), dim3(kSplatBlock), sa.lds.total, s,
                         (const int32_t*)L->stile_off.ptr, (const uint16_t*)L->run_rel.ptr,
                         (const int32_t*)L->run_dst.ptr, (const uint8_t*)L->ent_lp.ptr,
                         (const float*)L->ent_w.ptr, V, perm, part, pp, sa, *up);
    else
      hipLaunchKernelGGL((k_splat_tile<TU, G, false>), dim3(grid), dim3(kSplatBlock), sa.lds.total, s,
                         (const int32_t*)L->stile_off.ptr, (const uint16_t*)L->run_rel.ptr,
                         (const int32_t*)L->run_dst.ptr, (const uint8_t*)L->ent_lp.ptr,
                         (const float*)L->ent_w.ptr, V, perm, part, pp, sa, CgDirUpdate{});
    SGP_LAUNCH_CHECK("k_splat_tile");
  }
  {
    ProfScope ps(KK_SPLAT_GATHER, s);
    const int R = gather_rows(L);
    const int64_t ngroups = gather_ranges(L);
    constexpr int VWG = 16 / (int)sizeof(TU);  // channels per lane with 16-byte loads
    if (G % VWG == 0 && C % VWG == 0 && aligned16(part) && aligned16(U0) && aligned16(frag)) {
      const int64_t blocks = (ngroups + kBlock / (G / VWG) - 1) / (kBlock / (G / VWG));
      hipLaunchKernelGGL((k_splat_gather<TU, G, (G % VWG == 0 ? VWG : 1)>), dim3((unsigned)blocks), dim3(kBlock),
                         0, s, (const int32_t*)L->row_vert.ptr, part, U0, frag, L->npiece, C, ngroups, R);
    } else {
      const int64_t blocks = (ngroups + kBlock / G - 1) / (kBlock / G);
      hipLaunchKernelGGL((k_splat_gather<TU, G, 1>), dim3((unsigned)blocks), dim3(kBlock), 0, s,
                         (const int32_t*)L->row_vert.ptr, part, U0, frag, L->npiece, C, ngroups, R);
    }
    SGP_LAUNCH_CHECK("k_splat_gather");
    hipLaunchKernelGGL(k_gather_fix, dim3(grid_cap(ngroups * C)), dim3(kBlock), 0, s,
                       (const int32_t*)L->row_vert.ptr, (const int32_t*)L->occ_ptr.ptr, (const void*)frag,
                       (void*)U0, ngroups, C, (int)sizeof(TU), R);
    SGP_LAUNCH_CHECK("k_gather_fix");
  }

  const bool sym = L->blur == SGP_BLUR_SYMMETRIC;
  BlurArgs<TU> a;
  a.m = m;
  a.C = C;
  a.r = L->order;
  a.chains = sym ? 2 : 1;
  for (int t = 0; t < 2 * L->order + 1; ++t) a.st[t] = (TU)L->stencil64[t];
  unsigned bblocks;
  split_rows(m, kBlock / (G / blur_vw<G>()), 65536, &bblocks, &a.rows_per_block);
  a.vec = (C % Vec16<TU>::N == 0 && blur_vw<G>() % Vec16<TU>::N == 0 && aligned16(U0)) ? 1 : 0;
  // when the four lattice value arrays outgrow the 256 MiB Infinity Cache, the
  // blur's outputs stream past it, which keeps more of its inputs cached
  a.nt = (4.0 * (double)mC * sizeof(TU) > 256.0 * (1 << 20)) ? 1 : 0;
  const int32_t* nbr = (const int32_t*)L->nbr.ptr;
  // Chain 0 moves between B1 and B3 and never writes U0, which chain 1 reads
  // first; chain 1 moves between B2 and B4 (U0 outside CG). Steps run in
  // fused pairs when the stencil has three taps.
  const TU* cur[2] = {U0, U0};
  auto next0 = [&](const TU* c0) { return c0 == B1 ? B3 : B1; };
  auto next1 = [&](const TU* c1) { return c1 == B2 ? B4 : B2; };
  auto kdir = [&](int step, int chain) {
    return chain == 0 ? ((L->blur == SGP_BLUR_REVERSE) ? d - step : step) : d - step;
  };
  const bool fuse = L->order == 1 && blur_fuse_enabled();
  // Large lattices (the four value arrays over 128 MiB by default, half the
  // Infinity Cache): the chains' split launches run one chain after the
  // other (all of chain 0's, then chain 1's), so that a launch's input and
  // output arrays sit in the cache together.
  const bool seq = fuse && sym && blur_seq_for(4.0 * (double)mC * sizeof(TU));
  std::vector<Blur2Args<TU>> later;  // chain 1's split launches, in order
  auto launch2 = [&](const Blur2Args<TU>& b, unsigned grid) -> int {
    ProfScope ps(KK_BLUR, s);
    if (b.split)
      hipLaunchKernelGGL((k_blur2_split<TU, G>), dim3(grid), dim3(kBlock), 0, s, b);
    else
      hipLaunchKernelGGL((k_blur2<TU, G>), dim3(grid), dim3(kBlock), 0, s, b);
    SGP_LAUNCH_CHECK("k_blur2");
    return SGP_OK;
  };
  auto flush_later = [&]() -> int {
    for (const auto& b : later) {
      const int rc = launch2(b, bblocks);
      if (rc) return rc;
    }
    later.clear();
    return SGP_OK;
  };
  for (int step = 0; step <= d;) {
    TU* dst0 = next0(cur[0]);
    TU* dst1 = next1(cur[1]);
    if (fuse && step + 1 <= d) {
      Blur2Args<TU> b2;
      b2.in[0] = cur[0];
      b2.in[1] = cur[1];
      b2.out[0] = dst0;
      b2.out[1] = dst1;
      for (int ch = 0; ch < 2; ++ch) {
        b2.nbr1[ch] = nbr + (int64_t)kdir(step, ch) * T * m;
        b2.nbr2[ch] = nbr + (int64_t)kdir(step + 1, ch) * T * m;
      }
      b2.m = m;
      b2.C = C;
      b2.chains = a.chains;
      b2.sum_out = (sym && step + 1 == d) ? 1 : 0;
      b2.split = (a.chains == 2 && !b2.sum_out) ? 1 : 0;
      b2.chain0 = 0;
      b2.halves = 2;
      b2.vec = a.vec;
      b2.nt = a.nt;
      b2.rows_per_block = a.rows_per_block;
      for (int t = 0; t < 3; ++t) b2.st[t] = a.st[t];
      int rc;
      if (b2.split && seq) {
        b2.halves = 1;
        if ((rc = launch2(b2, bblocks))) return rc;
        b2.chain0 = 1;
        later.push_back(b2);
      } else {
        if ((rc = flush_later())) return rc;
        if ((rc = launch2(b2, b2.split ? 2 * bblocks : bblocks))) return rc;
      }
      step += 2;
    } else {
      a.in[0] = cur[0];
      a.out[0] = dst0;
      a.nbr[0] = nbr + (int64_t)kdir(step, 0) * T * m;
      a.in[1] = cur[1];
      a.out[1] = dst1;
      a.nbr[1] = nbr + (int64_t)kdir(step, 1) * T * m;
      a.sum_out = (sym && step == d) ? 1 : 0;
      if (const int rc = flush_later()) return rc;
      {
        ProfScope ps(KK_BLUR, s);
        hipLaunchKernelGGL((k_blur<TU, G>), dim3(bblocks), dim3(kBlock), 0, s, a);
        SGP_LAUNCH_CHECK("k_blur");
      }
      step += 1;
    }
    cur[0] = dst0;
    cur[1] = dst1;
  }
  if (const int rc = flush_later()) return rc;
  const TU scale = sym ? (TU)(0.5 * (double)L->outputscale) : (TU)L->outputscale;
  if (cgm) {
    // alpha from p.Ap = scale * u.(B u) + noise * p.p, before the slice
    const int rc = launch_cg_alpha((const double*)U0, (const double*)cur[0], m, C, (double)scale, *cgm, s);
    if (rc) return rc;
  }
  ProfScope ps(KK_SLICE, s);
  SliceArgs<TU> la;
  la.n = L->n;
  la.items = L->ntiles * chunks;
  la.P = P;
  la.D = D;
  la.C = C;
  la.chunks = chunks;
  la.cvec = (C % Vec16<TU>::N == 0 && aligned16(out) && (!p || aligned16(p))) ? 1 : 0;
  la.scale = scale;
  la.noise = noise;
  la.mrows = cgm ? L->solve_rows : 0;
  const int32_t* toff = (const int32_t*)L->tile_off.ptr;
  const int32_t* tverts = (const int32_t*)L->tile_verts.ptr;
  const uint16_t* loc = (const uint16_t*)L->loc.ptr;
  const float* ws = (const float*)L->ws.ptr;
  const uint32_t* mperm = (const uint32_t*)L->perm.ptr;
  auto launch = [&](auto nt_tag) {
    constexpr int NT = decltype(nt_tag)::value;
    la.lds = slice_lds<TU, G, NT>(P, D, maxq);
    if (cgm) {
      const unsigned grid = persistent_grid((const void*)&k_slice_tile<TU, G, true, NT>, NT, la.lds.total,
                                            la.items, lc.slice_bpc);
      hipLaunchKernelGGL((k_slice_tile<TU, G, true, NT>), dim3(grid), dim3(NT), la.lds.total, s, toff, tverts,
                         loc, ws, (const TU*)cur[0], out, perm, p, cgm->beta, mperm, la);
    } else {
      const unsigned grid = persistent_grid((const void*)&k_slice_tile<TU, G, false, NT>, NT, la.lds.total,
                                            la.items, lc.slice_bpc);
      hipLaunchKernelGGL((k_slice_tile<TU, G, false, NT>), dim3(grid), dim3(NT), la.lds.total, s, toff, tverts,
                         loc, ws, (const TU*)cur[0], out, perm, (const TU*)nullptr, CgHook{}, mperm, la);
    }
  };
  constexpr int NTn = slice_threads_narrow<G>();
  // the narrow block where the mean run list takes at most 2/3 of its pass
  if (NTn < 1024 && 3 * L->nrun <= 2 * L->ntiles * (int64_t)TileShape<TU, G, NTn>::RC)
    launch(std::integral_constant<int, NTn>{});
  else
    launch(std::integral_constant<int, 1024>{});
  SGP_LAUNCH_CHECK("k_slice_tile");
  return SGP_OK;
}

// Channel chunk: the widest power of two <= kMaxChunk covering C for which
// both tile kernels' LDS stages fit the budget. Chunks of at most 16
// channels stage whole blocks of kSliceOrderRows runs in the slice, so a
// column's results are the same bit for bit whatever the chunk; more
// columns take several chunks.
constexpr int kMaxChunk = 16;
int chunk_lanes(const sgp_lattice* L, int C, size_t elem) {
  int g = lanes_for(C);
  if (g > kMaxChunk) g = kMaxChunk;
  const int D = L->d + 1, P = L->tile_points, maxq = L->max_tile_runs, maxp = L->max_tile_pieces;
  const size_t budget = (size_t)tuning().lds_budget;
  const size_t slice_budget = (size_t)tuning().slice_lds_budget;
  while (g > 1) {
    const size_t splat = elem == 8 ? splat_lds<double>(P, D, maxp, g).total : splat_lds<float>(P, D, maxp, g).total;
    const size_t slice = elem == 8 ? slice_lds_g<double>(P, D, maxq, g) : slice_lds_g<float>(P, D, maxq, g);
    if (splat <= budget && slice <= slice_budget) break;
    g >>= 1;
  }
  return g;
}

// work: the MVM's work memory (mvm_work_elems(L, C, cgm) elements of TU),
// or null for the lattice's own buffer, grown on demand.
template <typename TU>
int mvm_dispatch(const sgp_lattice* L, const TU* V, const uint32_t* perm, int C, TU* out,
                 hipStream_t s, TU noise, const CgMvm* cgm, void* work = nullptr,
                 const CgDirUpdate* up = nullptr) {
  if (!work) {
    int rc = dev_reserve(L, const_cast<sgp_lattice*>(L)->ubuf,
                         sizeof(TU) * mvm_work_elems(L, C, cgm != nullptr), s);
    if (rc) return rc;
    work = L->ubuf.ptr;
  }
  const int gmax = chunk_lanes(L, C, sizeof(TU));
  LaunchChoice lc{gmax, 0, 0};
  if (g_force)
    lc = *g_force;
  else
    (void)tune_find(L, C, (int)sizeof(TU), &lc);
  if (lc.g < 1 || lc.g > gmax || (lc.g & (lc.g - 1))) lc.g = gmax;  // never wider than the LDS allows
  switch (lc.g) {
    case 1: return mvm_g<TU, 1>(L, V, perm, C, out, s, noise, cgm, lc, work, up);
    case 2: return mvm_g<TU, 2>(L, V, perm, C, out, s, noise, cgm, lc, work, up);
    case 4: return mvm_g<TU, 4>(L, V, perm, C, out, s, noise, cgm, lc, work, up);
    case 8: return mvm_g<TU, 8>(L, V, perm, C, out, s, noise, cgm, lc, work, up);
    default: return mvm_g<TU, 16>(L, V, perm, C, out, s, noise, cgm, lc, work, up);
  }
}

}  // namespace

int mvm_into(const sgp_lattice* L, const float* V, int C, float* out, hipStream_t s) {
  return mvm_dispatch<float>(L, V, (const uint32_t*)L->perm.ptr, C, out, s, 0.f, nullptr);
}

int mvm_cg(const sgp_lattice* L, double* p, int C, hipStream_t s, double noise, const CgMvm& cg,
           const CgDirUpdate* up) {
  return mvm_dispatch<double>(L, p, nullptr, C, cg.r, s, noise, &cg, nullptr, up);
}

int mvm_f64(const sgp_lattice* L, const double* V, int C, double* out, hipStream_t s) {
  return mvm_dispatch<double>(L, V, nullptr, C, out, s, 0.0, nullptr);
}

int mvm_f32(const sgp_lattice* L, const float* V, int C, float* out, hipStream_t s) {
  return mvm_dispatch<float>(L, V, nullptr, C, out, s, 0.f, nullptr);
}

// Times every candidate launch choice on this lattice and keeps the fastest
// for lattices of the same shape.
int autotune(const sgp_lattice* L, int C, bool fp64, int reps, hipStream_t s, int32_t* choice,
             float* best_ms) {
  const int elem = fp64 ? 8 : 4;
  const int gmax = chunk_lanes(L, C, elem);
  DevBuf buf;
  const size_t bytes = (size_t)elem * (size_t)L->n * (size_t)C;
  int rc = dev_alloc(buf, 2 * bytes, s);
  if (rc) return rc;
  struct Cleanup {
    DevBuf* b;
    hipStream_t s;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Cleanup() {
      g_force = nullptr;
      (void)hipStreamSynchronize(s);
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      dev_free(*b);
    }
  } cleanup{&buf, s};
  // values near 1 (every 32-bit word 0x3F800000 for fp32, 0x3FF00000 for fp64)
  if ((rc = launch_fill_u32((uint32_t*)buf.ptr, bytes / 4, fp64 ? 0x3FF00000u : 0x3F800000u, s))) return rc;
  SGP_HIP(hipEventCreate(&cleanup.e0));
  SGP_HIP(hipEventCreate(&cleanup.e1));
  void* V = buf.ptr;
  void* out = (char*)buf.ptr + bytes;
  auto run = [&]() {
    return fp64 ? mvm_f64(L, (const double*)V, C, (double*)out, s)
                : mvm_into(L, (const float*)V, C, (float*)out, s);
  };
  LaunchChoice best{gmax, 0, 0};
  float best_t = -1.f;
  for (int g = gmax; g >= 1 && g >= gmax / 4; g >>= 1) {
    for (int sb = 0; sb <= 1; ++sb) {
      for (int lb = 0; lb <= 1; ++lb) {
        const LaunchChoice cand{g, sb, lb};
        g_force = &cand;
        if ((rc = run())) return rc;  // warm-up (sizes buffers, sets LDS limits)
        SGP_HIP(hipEventRecord(cleanup.e0, s));
        for (int r = 0; r < reps; ++r)
          if ((rc = run())) return rc;
        SGP_HIP(hipEventRecord(cleanup.e1, s));
        SGP_HIP(hipEventSynchronize(cleanup.e1));
        float ms = 0.f;
        SGP_HIP(hipEventElapsedTime(&ms, cleanup.e0, cleanup.e1));
        ms /= (float)reps;
        if (best_t < 0.f || ms < best_t) {
          best_t = ms;
          best = cand;
        }
        g_force = nullptr;
      }
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const TuneEntry e{L->d, elem, lanes_for(C), mlog_of(L->m), best, best_t};
    bool found = false;
    for (TuneEntry& x : g_tune)
      if (x.d == e.d && x.elem == e.elem && x.g0 == e.g0 && x.mlog == e.mlog) {
        x = e;
        found = true;
      }
    if (!found) g_tune.push_back(e);
  }
  if (choice) {
    choice[0] = best.g;
    choice[1] = best.splat_bpc;
    choice[2] = best.slice_bpc;
  }
  if (best_ms) *best_ms = best_t;
  mark_use(L, s);
  return SGP_OK;
}

void autotune_reset() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
}

}  // namespace sgp

using namespace sgp;

extern "C" int lattice_mvm(const sgp_lattice* L, const float* values, int32_t C, float* out,
                           void* stream) {
  if (!L || !values || !out) {
    set_error("lattice_mvm: NULL argument");
    return SGP_EINVAL;
  }
  if (C < 1) {
    set_error("lattice_mvm: C must be >= 1 (got %d)", (int)C);
    return SGP_EINVAL;
  }
  const size_t bytes = sizeof(float) * (size_t)L->n * (size_t)C;
  const char* v0 = (const char*)values;
  const char* o0 = (const char*)out;
  if (v0 < o0 + bytes && o0 < v0 + bytes) {
    set_error("lattice_mvm: out overlaps values");
    return SGP_EINVAL;
  }
  const int rc = mvm_into(L, values, C, out, (hipStream_t)stream);
  if (rc == SGP_OK) mark_use(L, (hipStream_t)stream);
  return rc;
}

// Work memory of lattice_mvm_noalloc: one array per device, part of the
// code object, held until the process ends. In host code `scratch` names a
// host-side stand-in, not device memory: kernels receive the device address
// that hipGetSymbolAddress returns for the current device, looked up once per
// device on its first call.
namespace {
constexpr size_t kScratchBytes = (size_t)SGP_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kScratchDevices] = {};

int scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      set_error("lattice_mvm_noalloc: no device address for the scratch array on device %d: %s", dev,
                hipGetErrorString(e));
      return SGP_EHIP;
    }
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return SGP_OK;
}
}  // namespace

extern "C" int lattice_mvm_noalloc(const sgp_lattice* L, const float* values, int32_t C, float* out,
                                   void* stream) {
  if (!L || !values || !out) {
    set_error("lattice_mvm_noalloc: NULL argument");
    return SGP_EINVAL;
  }
  if (C < 1) {
    set_error("lattice_mvm_noalloc: C must be >= 1 (got %d)", (int)C);
    return SGP_EINVAL;
  }
  const size_t bytes = sizeof(float) * (size_t)L->n * (size_t)C;
  const char* v0 = (const char*)values;
  const char* o0 = (const char*)out;
  if (v0 < o0 + bytes && o0 < v0 + bytes) {
    set_error("lattice_mvm_noalloc: out overlaps values");
    return SGP_EINVAL;
  }
  const size_t need = sizeof(float) * mvm_work_elems(L, C, false);
  if (need > kScratchBytes) {
    set_error("lattice_mvm_noalloc: this lattice and C = %d need %zu bytes of work memory; the "
              "no-allocation entry point has %zu (use lattice_mvm)", (int)C, need, kScratchBytes);
    return SGP_EINVAL;
  }
  int dev = 0;
  SGP_HIP(hipGetDevice(&dev));
  if (dev != L->device || dev < 0 || dev >= kScratchDevices) {
    set_error("lattice_mvm_noalloc: make the lattice's device (%d) current (current: %d)", L->device, dev);
    return SGP_EINVAL;
  }
  void* work = nullptr;
  int rc = scratch_address(dev, &work);
  if (rc) return rc;
  rc = mvm_dispatch<float>(L, values, (const uint32_t*)L->perm.ptr, C, out, (hipStream_t)stream, 0.f,
                           nullptr, work);
  if (rc == SGP_OK) mark_use(L, (hipStream_t)stream);
  return rc;
}

extern "C" int sgp_autotune(const sgp_lattice* L, int32_t C, int32_t fp64, int32_t reps, void* stream,
                            int32_t* choice, float* ms_per_mvm) {
  if (!L) {
    set_error("sgp_autotune: NULL lattice");
    return SGP_EINVAL;
  }
  if (C < 1 || (fp64 && C > kMaxCgCols) || reps < 1) {
    set_error("sgp_autotune: need C >= 1 (at most %d in fp64) and reps >= 1", kMaxCgCols);
    return SGP_EINVAL;
  }
  return autotune(L, C, fp64 != 0, reps, (hipStream_t)stream, choice, ms_per_mvm);
}

extern "C" int sgp_autotune_reset(void) {
  autotune_reset();
  build_tune_reset();
  return SGP_OK;
}
