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
// Channels are processed in chunks of G (a power of two <= 64) chosen so
// that the staged rows fit the LDS budget; chunks are the grid's y axis.
// Row ranges of consecutive blocks go to the same XCD (blocks are dealt
// round-robin over the 8 XCDs), so tiles that share lattice points share
// an L2.
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

// LDS layout of k_splat_tile: values [P][G] (TU) | weights [P*D] (fp32) |
// run starts [runs+1] (uint16) | entry points [P*D] (uint8).
template <typename TU>
__host__ __device__ inline size_t splat_lds_bytes(int P, int D, int runs, int G, bool stage_v) {
  size_t b = stage_v ? sizeof(TU) * (size_t)P * G : 0;
  b += sizeof(float) * (size_t)P * D;
  b += sizeof(uint16_t) * (size_t)(runs + 1);
  b = (b + 3) & ~(size_t)3;
  b += (size_t)P * D;
  return (b + 15) & ~(size_t)15;
}

// Copy a tile's n (<= kMaxTileEntries) entries (weight + small index) to
// LDS with every load of the thread issued before its stores.
constexpr int kMaxTileEntries = 4096;
template <typename IDX>
__device__ __forceinline__ void stage_entries(const float* __restrict__ w, const IDX* __restrict__ ix,
                                              int n, float* lw, IDX* lix) {
  constexpr int kPer = kMaxTileEntries / kBlock;
  float wt[kPer];
  IDX it[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int i = threadIdx.x + u * kBlock;
    if (i < n) {
      wt[u] = w[i];
      it[u] = ix[i];
    }
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int i = threadIdx.x + u * kBlock;
    if (i < n) {
      lw[i] = wt[u];
      lix[i] = it[u];
    }
  }
}

template <typename TV, typename TU, int G>
__global__ __launch_bounds__(kBlock) void k_splat_tile(const int32_t* __restrict__ tile_off,
                                                       const uint16_t* __restrict__ run_rel,
                                                       const uint8_t* __restrict__ ent_lp,
                                                       const float* __restrict__ ent_w,
                                                       const TV* __restrict__ V,
                                                       const uint32_t* __restrict__ perm,
                                                       TU* __restrict__ part, int64_t n, int P, int D,
                                                       int C, int stage_v) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int R = kBlock / G;
  const int lane = threadIdx.x % G, row = threadIdx.x / G;
  const int64_t t = blockIdx.x;
  const int c = blockIdx.y * G + lane;
  const bool cv = c < C;
  const int64_t p0 = t * P;
  const int np = (int)(n - p0 < P ? n - p0 : P);
  const int ne = np * D;
  const int64_t ebase = p0 * D;
  const int q0 = tile_off[t], nq = tile_off[t + 1] - q0;
  TU* lv = (TU*)smem;
  float* lw = (float*)(lv + (size_t)(stage_v ? P : 0) * G);
  uint16_t* lrel = (uint16_t*)(lw + (size_t)P * D);
  uint8_t* llp = (uint8_t*)(((uintptr_t)(lrel + nq + 1) + 3) & ~(uintptr_t)3);
  // stage the tile: its points' values, its entries and its run starts.
  // Every load of a thread is issued before any LDS store, so the loads of
  // one thread are in flight together.
  if (stage_v) {
    // np <= P <= R * G: at most G rows per thread
    TU vt[G];
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int lp = row + i * R;
      vt[i] = 0;
      if (lp < np && cv) {
        const int64_t pt = p0 + lp;
        const int64_t src = perm ? (int64_t)perm[pt] : pt;
        vt[i] = (TU)V[src * C + c];
      }
    }
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int lp = row + i * R;
      if (lp < np) lv[lp * G + lane] = vt[i];
    }
  }
  stage_entries(ent_w + ebase, ent_lp + ebase, ne, lw, llp);
  for (int i = threadIdx.x; i < nq; i += kBlock) lrel[i] = run_rel[q0 + i];
  if (threadIdx.x == 0) lrel[nq] = (uint16_t)ne;
  __syncthreads();
  // one run (= one lattice point of this tile) per G lanes, entries in order
  for (int qq = row; qq < nq; qq += R) {
    TU acc = 0;
    const int e1 = lrel[qq + 1];
    if (stage_v) {
      int e = lrel[qq];
      for (; e + 4 <= e1; e += 4) {
        int lp[4];
        float wv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          lp[u] = llp[e + u];
          wv[u] = lw[e + u];
        }
        TU v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = lv[lp[u] * G + lane];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = fma_t((TU)wv[u], v[u], acc);
      }
      for (; e < e1; ++e) acc = fma_t((TU)lw[e], lv[(int)llp[e] * G + lane], acc);
    } else if (cv) {
      for (int e = lrel[qq]; e < e1; ++e) {
        const int64_t pt = p0 + llp[e];
        const int64_t src = perm ? (int64_t)perm[pt] : pt;
        acc = fma_t((TU)lw[e], (TU)V[src * C + c], acc);
      }
    }
    if (cv) part[(int64_t)(q0 + qq) * C + c] = acc;
  }
}

// Lattice point j sums its partial rows; S = G*E lanes per point, E lanes
// striding its list, combined by a fixed butterfly.
template <typename TU, int G>
__global__ __launch_bounds__(kBlock) void k_splat_gather(const int32_t* __restrict__ occ_ptr,
                                                         const int32_t* __restrict__ occ,
                                                         const TU* __restrict__ part,
                                                         TU* __restrict__ U, int64_t m, int C, int E,
                                                         int64_t rows_per_block) {
  const int S = G * E;
  const int gl = threadIdx.x % S;
  const int c0 = gl % G, u = gl / G;
  const int groups = kBlock / S;
  const int64_t j0 = xcd_block(blockIdx.x, gridDim.x) * rows_per_block;
  const int64_t j1 = j0 + rows_per_block < m ? j0 + rows_per_block : m;
  for (int64_t j = j0 + threadIdx.x / S; j < j1; j += groups) {
    const int o0 = occ_ptr[j], o1 = occ_ptr[j + 1];
    for (int c = c0; c < C; c += G) {
      TU acc = 0;
      for (int o = o0 + u; o < o1; o += E) acc += part[(int64_t)occ[o] * C + c];
      for (int off = G; off < S; off <<= 1) acc += __shfl_xor(acc, off);
      if (u == 0) U[j * C + c] = acc;
    }
  }
}

template <typename TU>
struct BlurArgs {
  const TU* in[2];
  TU* out[2];
  const int32_t* nbr[2];  // neighbour table of this step's direction, per chain
  int64_t m;
  int C;
  int r;
  int chains;
  int sum_out;  // last SYMMETRIC step: out[0] = forward + reverse
  int64_t rows_per_block;
  TU st[2 * kMaxOrder + 1];
};

template <typename TU>
__device__ __forceinline__ TU blur_row(const TU* __restrict__ in, const int32_t* __restrict__ nb,
                                       int64_t m, int64_t j, int C, int c, int r, const TU* st) {
  TU acc = 0;
  int ti = 0;
  for (int t = -r; t <= r; ++t) {
    TU v;
    if (t == 0) {
      v = in[j * C + c];
    } else {
      const int32_t x = nb[(int64_t)ti * m + j];
      v = x >= 0 ? in[(int64_t)x * C + c] : (TU)0;
      ++ti;
    }
    acc = fma_t(st[t + r], v, acc);
  }
  return acc;
}

template <typename TU, int G>
__global__ __launch_bounds__(kBlock) void k_blur(BlurArgs<TU> a) {
  constexpr int R = kBlock / G;
  const int lane = threadIdx.x % G;
  const int64_t j0 = xcd_block(blockIdx.x, gridDim.x) * a.rows_per_block;
  const int64_t j1 = j0 + a.rows_per_block < a.m ? j0 + a.rows_per_block : a.m;
  for (int64_t j = j0 + threadIdx.x / G; j < j1; j += R) {
    for (int c = lane; c < a.C; c += G) {
      const TU f = blur_row(a.in[0], a.nbr[0], a.m, j, a.C, c, a.r, a.st);
      if (a.chains == 2) {
        const TU b = blur_row(a.in[1], a.nbr[1], a.m, j, a.C, c, a.r, a.st);
        if (a.sum_out) {
          a.out[0][j * a.C + c] = f + b;
        } else {
          a.out[0][j * a.C + c] = f;
          a.out[1][j * a.C + c] = b;
        }
      } else {
        a.out[0][j * a.C + c] = f;
      }
    }
  }
}

// LDS layout of k_slice_tile: lattice rows [RC][G] (TU) | weights [P*D]
// (fp32) | slots [P*D] (uint16).
template <typename TU>
__host__ __device__ inline size_t slice_lds_bytes(int P, int D, int RC, int G) {
  size_t b = sizeof(TU) * (size_t)RC * G;
  if (b < sizeof(double) * kBlock) b = sizeof(double) * kBlock;  // CG reduction reuses it
  b += sizeof(float) * (size_t)P * D;
  b += sizeof(uint16_t) * (size_t)P * D;
  return (b + 15) & ~(size_t)15;
}

// The tile's (slot, weight) entries are staged once; its lattice rows are
// staged RC at a time, and each point adds the entries whose slot falls in
// the staged chunk. A thread keeps the sums of its ceil(P/R) <= G points.
template <typename TV, typename TU, int G, bool CG>
__global__ __launch_bounds__(kBlock) void k_slice_tile(const int32_t* __restrict__ tile_off,
                                                       const int32_t* __restrict__ tile_verts,
                                                       const uint16_t* __restrict__ loc,
                                                       const float* __restrict__ ws,
                                                       const TU* __restrict__ U,
                                                       TV* __restrict__ out,
                                                       const uint32_t* __restrict__ perm, int64_t n,
                                                       int P, int D, int C, int RC, TU scale, TV noise,
                                                       const TV* __restrict__ p,
                                                       double* __restrict__ partials,
                                                       const uint32_t* __restrict__ mperm,
                                                       int64_t mrows) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int R = kBlock / G;
  const int lane = threadIdx.x % G, row = threadIdx.x / G;
  const int64_t t = xcd_block(blockIdx.x, gridDim.x);
  const int c = blockIdx.y * G + lane;
  const bool cv = c < C;
  const int64_t p0 = t * P;
  const int np = (int)(n - p0 < P ? n - p0 : P);
  const int ne = np * D;
  const int64_t ebase = p0 * D;
  const int q0 = tile_off[t], nq = tile_off[t + 1] - q0;
  size_t ub = sizeof(TU) * (size_t)RC * G;
  if (ub < sizeof(double) * kBlock) ub = sizeof(double) * kBlock;
  TU* lu = (TU*)smem;
  float* lw = (float*)(smem + ub);
  uint16_t* lsl = (uint16_t*)(lw + (size_t)P * D);
  stage_entries(ws + ebase, loc + ebase, ne, lw, lsl);
  TU acc[G];
#pragma unroll
  for (int a = 0; a < G; ++a) acc[a] = 0;
  for (int r0 = 0; r0 < nq; r0 += RC) {
    const int nr = nq - r0 < RC ? nq - r0 : RC;
    __syncthreads();  // previous chunk fully consumed (and entries staged)
    // eight rows per thread in flight: indices first, then the rows
    for (int sb = row; sb < nr; sb += 8 * R) {
      int32_t vj[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int sr = sb + u * R;
        vj[u] = sr < nr ? tile_verts[q0 + r0 + sr] : 0;
      }
      TU vr[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int sr = sb + u * R;
        vr[u] = (sr < nr && cv) ? U[(int64_t)vj[u] * C + c] : (TU)0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int sr = sb + u * R;
        if (sr < nr) lu[sr * G + lane] = vr[u];
      }
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < G; ++a) {
      const int lp = a * R + row;
      if (lp < np) {
        const int eb = lp * D;
        int k = 0;
        for (; k + 4 <= D; k += 4) {
          int sl[4];
          float wv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            sl[u] = (int)lsl[eb + k + u] - r0;
            wv[u] = lw[eb + k + u];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if ((unsigned)sl[u] < (unsigned)nr) acc[a] = fma_t((TU)wv[u], lu[sl[u] * G + lane], acc[a]);
        }
        for (; k < D; ++k) {
          const int sl = (int)lsl[eb + k] - r0;
          if ((unsigned)sl < (unsigned)nr) acc[a] = fma_t((TU)lw[eb + k], lu[sl * G + lane], acc[a]);
        }
      }
    }
  }
  double dot = 0.0;
#pragma unroll
  for (int a = 0; a < G; ++a) {
    const int lp = a * R + row;
    if (lp < np && cv) {
      const int64_t pt = p0 + lp;
      TV o = (TV)(scale * acc[a]);
      if (CG) {
        const TV pv = p[pt * C + c];
        o = fma_t(noise, pv, o);
        if (mrows > 0 && (int64_t)mperm[pt] >= mrows) o = 0;  // not solved for
        dot += (double)pv * (double)o;
      }
      out[(perm ? (int64_t)perm[pt] : pt) * C + c] = o;
    }
  }
  if (CG) {
    __syncthreads();
    double* sh = (double*)smem;
    sh[threadIdx.x] = dot;
    __syncthreads();
    if ((int)threadIdx.x < G && cv) {
      double s = 0.0;
      for (int rr = 0; rr < R; ++rr) s += sh[rr * G + threadIdx.x];
      partials[t * C + c] = s;
    }
  }
}

int slice_rows_per_chunk(const sgp_lattice* L, int G, size_t elem);

// Blocks for `rows` rows at R per block, capped, and the rows each block
// takes so that the blocks cover all rows.
void split_rows(int64_t rows, int R, int64_t cap, unsigned* blocks, int64_t* rows_per_block) {
  int64_t b = (rows + R - 1) / R;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  *rows_per_block = (rows + b - 1) / b;
  *blocks = (unsigned)((rows + *rows_per_block - 1) / *rows_per_block);
}

template <typename TV, typename TU, int G>
int mvm_g(const sgp_lattice* L, const TV* V, const uint32_t* perm, int C, TV* out, hipStream_t s,
          TV noise, const TV* p, double* partials) {
  const int d = L->d, D = d + 1, T = 2 * L->order;
  const int64_t m = L->m, mC = m * C;
  TU* U0 = (TU*)L->ubuf.ptr;
  TU* B1 = U0 + mC;
  TU* B2 = B1 + mC;
  TU* B3 = B2 + mC;
  TU* part = B3 + mC;
  const int chunks = (C + G - 1) / G;
  const int P = L->tile_points;
  const dim3 tgrid((unsigned)L->ntiles, (unsigned)chunks);
  {
    ProfScope ps(KK_SPLAT, s);
    const bool stage_v = tuning().splat_stage_v != 0;
    const size_t lds = splat_lds_bytes<TU>(P, D, L->max_tile_runs, G, stage_v);
    hipLaunchKernelGGL((k_splat_tile<TV, TU, G>), tgrid, dim3(kBlock), lds, s,
                       (const int32_t*)L->tile_off.ptr, (const uint16_t*)L->run_rel.ptr,
                       (const uint8_t*)L->ent_lp.ptr, (const float*)L->ent_w.ptr, V, perm, part, L->n,
                       P, D, C, stage_v ? 1 : 0);
    SGP_LAUNCH_CHECK("k_splat_tile");
  }
  {
    ProfScope ps(KK_SPLAT_GATHER, s);
    // lanes per point's list: about a quarter of its mean length
    const double avg = (double)L->nrun / (double)m;
    int E = 1;
    while (E * 2 * G <= 64 && E * 2 <= avg / 4.0) E *= 2;
    unsigned blocks;
    int64_t rpb;
    split_rows(m, kBlock / (G * E), 65536, &blocks, &rpb);
    hipLaunchKernelGGL((k_splat_gather<TU, G>), dim3(blocks), dim3(kBlock), 0, s,
                       (const int32_t*)L->occ_ptr.ptr, (const int32_t*)L->occ.ptr, part, U0, m, C, E,
                       rpb);
    SGP_LAUNCH_CHECK("k_splat_gather");
  }

  const bool sym = L->blur == SGP_BLUR_SYMMETRIC;
  BlurArgs<TU> a;
  a.m = m;
  a.C = C;
  a.r = L->order;
  a.chains = sym ? 2 : 1;
  for (int t = 0; t < 2 * L->order + 1; ++t) a.st[t] = (TU)L->stencil64[t];
  unsigned bblocks;
  split_rows(m, kBlock / G, 65536, &bblocks, &a.rows_per_block);
  const int32_t* nbr = (const int32_t*)L->nbr.ptr;
  const TU* cur[2] = {U0, U0};
  for (int step = 0; step <= d; ++step) {
    // chain 0: forward (or the single requested order); chain 1: reverse
    const int k0 = (L->blur == SGP_BLUR_REVERSE) ? d - step : step;
    const int k1 = d - step;
    TU* dst0 = (step % 2 == 0) ? B1 : B3;
    TU* dst1 = (step % 2 == 0) ? B2 : U0;
    a.in[0] = cur[0];
    a.out[0] = dst0;
    a.nbr[0] = nbr + (int64_t)k0 * T * m;
    a.in[1] = cur[1];
    a.out[1] = dst1;
    a.nbr[1] = nbr + (int64_t)k1 * T * m;
    a.sum_out = (sym && step == d) ? 1 : 0;
    {
      ProfScope ps(KK_BLUR, s);
      hipLaunchKernelGGL((k_blur<TU, G>), dim3(bblocks), dim3(kBlock), 0, s, a);
      SGP_LAUNCH_CHECK("k_blur");
    }
    cur[0] = dst0;
    cur[1] = dst1;
  }
  const TU scale = sym ? (TU)(0.5 * (double)L->outputscale) : (TU)L->outputscale;
  ProfScope ps(KK_SLICE, s);
  const int RC = slice_rows_per_chunk(L, G, sizeof(TU));
  const size_t lds = slice_lds_bytes<TU>(P, D, RC, G);
  if (partials) {
    hipLaunchKernelGGL((k_slice_tile<TV, TU, G, true>), tgrid, dim3(kBlock), lds, s,
                       (const int32_t*)L->tile_off.ptr, (const int32_t*)L->tile_verts.ptr,
                       (const uint16_t*)L->loc.ptr, (const float*)L->ws.ptr, cur[0], out, perm,
                       L->n, P, D, C, RC, scale, noise, p, partials, (const uint32_t*)L->perm.ptr,
                       L->solve_rows);
  } else {
    hipLaunchKernelGGL((k_slice_tile<TV, TU, G, false>), tgrid, dim3(kBlock), lds, s,
                       (const int32_t*)L->tile_off.ptr, (const int32_t*)L->tile_verts.ptr,
                       (const uint16_t*)L->loc.ptr, (const float*)L->ws.ptr, cur[0], out, perm,
                       L->n, P, D, C, RC, scale, (TV)0, (const TV*)nullptr, nullptr,
                       (const uint32_t*)nullptr, (int64_t)0);
  }
  SGP_LAUNCH_CHECK("k_slice_tile");
  return SGP_OK;
}

// Lattice rows per staged chunk in the slice: what the LDS budget leaves
// after the tile's entries, at most the longest run list.
int slice_rows_per_chunk(const sgp_lattice* L, int G, size_t elem) {
  const size_t ent = (sizeof(float) + sizeof(uint16_t)) * (size_t)L->tile_points * (L->d + 1);
  const size_t budget = (size_t)tuning().lds_budget;
  const size_t room = budget > ent ? budget - ent : 0;
  int64_t rc = (int64_t)(room / (elem * G));
  if (rc > L->max_tile_runs) rc = L->max_tile_runs;
  if (tuning().slice_rows > 0 && rc > tuning().slice_rows) rc = tuning().slice_rows;
  return rc < 1 ? 1 : (int)rc;
}

// Channel chunk: the widest power of two <= 64 covering C for which the
// splat's staged tile fits the LDS budget and the slice stages at least 64
// lattice rows (or all of a tile's rows) per chunk.
int chunk_lanes(const sgp_lattice* L, int C, size_t elem) {
  int g = lanes_for(C);
  const int D = L->d + 1, P = L->tile_points;
  while (g > 1) {
    const bool sv = tuning().splat_stage_v != 0;
    const size_t splat = elem == 8 ? splat_lds_bytes<double>(P, D, L->max_tile_runs, g, sv)
                                   : splat_lds_bytes<float>(P, D, L->max_tile_runs, g, sv);
    const int rc = slice_rows_per_chunk(L, g, elem);
    if (splat <= (size_t)tuning().lds_budget && (rc >= 64 || rc >= L->max_tile_runs)) break;
    g >>= 1;
  }
  return g;
}

template <typename TV, typename TU>
int mvm_dispatch(const sgp_lattice* L, const TV* V, const uint32_t* perm, int C, TV* out,
                 hipStream_t s, TV noise, const TV* p, double* partials) {
  int rc = dev_reserve(L, const_cast<sgp_lattice*>(L)->ubuf,
                       sizeof(TU) * (4 * L->m + L->nrun) * (size_t)C, s);
  if (rc) return rc;
  switch (chunk_lanes(L, C, sizeof(TU))) {
    case 1: return mvm_g<TV, TU, 1>(L, V, perm, C, out, s, noise, p, partials);
    case 2: return mvm_g<TV, TU, 2>(L, V, perm, C, out, s, noise, p, partials);
    case 4: return mvm_g<TV, TU, 4>(L, V, perm, C, out, s, noise, p, partials);
    case 8: return mvm_g<TV, TU, 8>(L, V, perm, C, out, s, noise, p, partials);
    case 16: return mvm_g<TV, TU, 16>(L, V, perm, C, out, s, noise, p, partials);
    case 32: return mvm_g<TV, TU, 32>(L, V, perm, C, out, s, noise, p, partials);
    default: return mvm_g<TV, TU, 64>(L, V, perm, C, out, s, noise, p, partials);
  }
}

}  // namespace

int mvm_into(const sgp_lattice* L, const float* V, int C, float* out, hipStream_t s) {
  return mvm_dispatch<float, float>(L, V, (const uint32_t*)L->perm.ptr, C, out, s, 0.f, nullptr,
                                    nullptr);
}

int mvm_cg(const sgp_lattice* L, const double* p, int C, double* q, hipStream_t s, double noise,
           double* partials) {
  return mvm_dispatch<double, double>(L, p, nullptr, C, q, s, noise, p, partials);
}

int mvm_f64(const sgp_lattice* L, const double* V, int C, double* out, hipStream_t s) {
  return mvm_dispatch<double, double>(L, V, nullptr, C, out, s, 0.0, nullptr, nullptr);
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
