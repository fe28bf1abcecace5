// Conjugate gradients on (outputscale*K + noise*I) x = b, one independent
// recurrence per column (Section 2, Krylov methods; Section 5.4 on
// tolerances). All scalars stay on the device. Each iteration is one
// lattice MVM that finishes the step itself: its splat applies the previous
// direction update and emits p.p per tile; after the blur a lattice kernel
// forms p.Ap = scale * u.(B u) + noise * p.p (u = W^T p: the quadratic
// form of W B W^T taken on the m lattice rows instead of the n points) and
// a one-block kernel turns it into alpha; the slice then moves the residual
// (r -= alpha A p, never storing A p) and its last block decides
// convergence and beta. The host only polls the per-column "active" flags
// every few iterations.
//
// Precision: the recurrence vectors (r, p), the lattice values inside
// its MVMs and all reductions are fp64; the barycentric weights and x stay
// fp32 (x is only accumulated, each update formed in fp64 and rounded once).
// With an fp32 recurrence the recursive residual drifts from the true one by
// about eps * cond(A), which at the conditioning of typical GP systems
// (cond ~ 1e3..1e4) is already above a 1e-4 tolerance. The caller's rhs and
// x are fp32. Partial sums are reduced in a fixed order, so a run is
// reproducible given the MVM's own rounding.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "cg_step.h"
#include "sgp_internal.h"

namespace sgp {
namespace {

// Vectors live in the lattice's internal point order: b is gathered through
// the permutation here and x scattered back in k_cg_out.
// The vector kernels give one partial sum per column for every superchunk of
// S chunks of kCgChunk rows. A chunk is 16 groups of 8 rows, each group added
// in row order, then the 16 group sums in order; a superchunk adds its chunk
// sums in order. The order depends on the rows only, not on how many columns
// are solved together, so a column's iterates are the same alone or in a
// batch. A block takes a superchunk at a time, kCpb(C) chunks per pass;
// thread (chunk, group, column) has the column fastest, so the threads of a
// group read whole rows. The init kernel uses S = 1 over the points, which
// gives it more blocks for its gathered loads; the alpha kernel S = 2 over
// the lattice rows.
constexpr int kCgChunk = 128;
constexpr int kCgGroups = 16;
constexpr int kCgRowsPerGroup = kCgChunk / kCgGroups;
constexpr int kSuperLat = 2;
constexpr int kSuperInit = 1;
__host__ __device__ inline int64_t cg_chunks(int64_t n) { return (n + kCgChunk - 1) / kCgChunk; }
__host__ __device__ inline int64_t cg_supers(int64_t n, int S) { return (cg_chunks(n) + S - 1) / S; }
__host__ __device__ inline int cg_cpb(int C) {
  const int per = kCgGroups * C;
  return per >= kBlock ? 1 : kBlock / per;
}
// Dynamic LDS of a vector kernel: the group sums of one pass.
inline size_t cg_vec_lds(int C) { return sizeof(double) * (size_t)(cg_cpb(C) * kCgGroups * C); }

// Runs gsum(first row, column) for every group of the block's superchunks
// and writes one partial per superchunk and column.
template <int S, typename GroupSum>
__device__ inline void cg_partials(int64_t n, int C, double* __restrict__ partials, double* sh,
                                   GroupSum gsum) {
  const int cpb = cg_cpb(C);
  const int64_t nchunks = cg_chunks(n), nsup = cg_supers(n, S);
  for (int64_t sup = blockIdx.x; sup < nsup; sup += gridDim.x) {
    const int64_t c0 = sup * S;
    const int64_t c1 = c0 + S < nchunks ? c0 + S : nchunks;
    double acc = 0.0;  // thread c < C: column c's superchunk sum so far
    for (int64_t chunk0 = c0; chunk0 < c1; chunk0 += cpb) {
      const int nck = (int)(c1 - chunk0 < cpb ? c1 - chunk0 : cpb);
      for (int q = threadIdx.x; q < nck * kCgGroups * C; q += blockDim.x) {
        const int c = q % C, gq = q / C;  // gq = chunk * groups + group
        sh[q] = gsum((chunk0 + gq / kCgGroups) * kCgChunk + (gq % kCgGroups) * kCgRowsPerGroup, c);
      }
      __syncthreads();
      if ((int)threadIdx.x < C) {
        for (int ck = 0; ck < nck; ++ck) {
          double v = 0.0;
          for (int g = 0; g < kCgGroups; ++g) v += sh[(ck * kCgGroups + g) * C + threadIdx.x];
          acc += v;
        }
      }
      __syncthreads();
    }
    if ((int)threadIdx.x < C) partials[sup * C + threadIdx.x] = acc;
  }
}

// x = 0, r = p = b (rows at or past `rows` zero when rows > 0), and the
// starting r.r.
__global__ __launch_bounds__(kBlock) void k_cg_init(const float* __restrict__ b,
                                                    const uint32_t* __restrict__ perm,
                                                    float* __restrict__ x,
                                                    double* __restrict__ r, double* __restrict__ p,
                                                    int64_t n, int C, int64_t rows,
                                                    double* __restrict__ partials) {
  extern __shared__ double dsh[];
  cg_partials<kSuperInit>(n, C, partials, dsh, [=](int64_t i0, int c) {
    // all loads of the group first, then the stores
    uint32_t src[kCgRowsPerGroup];
    double v[kCgRowsPerGroup];
#pragma unroll
    for (int k = 0; k < kCgRowsPerGroup; ++k) src[k] = i0 + k < n ? perm[i0 + k] : 0u;
#pragma unroll
    for (int k = 0; k < kCgRowsPerGroup; ++k)
      v[k] = (i0 + k < n && !(rows > 0 && src[k] >= rows)) ? (double)b[(int64_t)src[k] * C + c] : 0.0;
    double dot = 0.0;
#pragma unroll
    for (int k = 0; k < kCgRowsPerGroup; ++k) {
      if (i0 + k < n) {
        const int64_t e = (i0 + k) * C + c;
        x[e] = 0.0f;
        r[e] = v[k];
        p[e] = v[k];
        dot += v[k] * v[k];
      }
    }
    return dot;
  });
}

// Partial sums of p.Ap for alpha. Blocks [0, lat_parts) take one
// superchunk of lattice rows each: scale * u.(B u) per column (the
// quadratic form p.(scale K) p). Block lat_parts + g adds tile rows
// 16g .. 16g + 15 of the splat's noise * p.p in order. All of these rows
// are then folded into p.Ap and alpha (the order depends on m and the tile
// count only): by the last block to finish when the kernel has few blocks
// (fold), else by k_cg_scalar, as a device-scope fence in every one of
// thousands of blocks costs more than the launch.
constexpr int64_t kAlphaFoldBlocks = 256;
__global__ __launch_bounds__(kBlock) void k_cg_alpha(const double* __restrict__ u,
                                                     const double* __restrict__ bu, int64_t m, int C,
                                                     double scale, int64_t lat_parts,
                                                     const double* __restrict__ pp, int64_t ntiles,
                                                     CgHook h, int fold) {
  extern __shared__ double dsh[];
  cg_partials<kSuperLat>(m, C, h.partials, dsh, [=](int64_t i0, int c) {
    double uv[kCgRowsPerGroup], bv[kCgRowsPerGroup];
#pragma unroll
    for (int k = 0; k < kCgRowsPerGroup; ++k) {
      const int64_t e = (i0 + k < m ? i0 + k : m - 1) * C + c;
      uv[k] = u[e];
      bv[k] = bu[e];
    }
    double dot = 0.0;
#pragma unroll
    for (int k = 0; k < kCgRowsPerGroup; ++k)
      if (i0 + k < m) dot = __builtin_fma(uv[k], bv[k], dot);
    return scale * dot;
  });
  const int64_t g = (int64_t)blockIdx.x - lat_parts;
  if (g >= 0) {
    const int64_t t0 = g * 16, t1 = t0 + 16 < ntiles ? t0 + 16 : ntiles;
    for (int c = threadIdx.x; c < C; c += blockDim.x) {
      double v = 0.0;
      for (int64_t t = t0; t < t1; ++t) v += pp[t * C + c];
      h.partials[(lat_parts + g) * C + c] = v;
    }
  }
  if (fold) cg_finish(h, C, dsh);
}

// The scalar step after a vector kernel, in one block of its own: the
// kernel boundary makes every block's partials visible at the cost of one
// L2 writeback per XCD, where a last-block fold inside a kernel of
// thousands of blocks would pay one per block.
constexpr int kScalarThreads = 1024;
__global__ __launch_bounds__(kScalarThreads) void k_cg_scalar(CgHook h, int C) {
  __shared__ double sh[kFold * kMaxCgCols];
  cg_scalar_block(h.partials, h.nparts, C, h.st, h.mode, h.tol, sh);
}

// x += alpha p with this iteration's alpha (zero for a column that was
// already converged), then p = r + beta p for the columns still active.
// Element-wise over the n x C arrays, two elements (one 16-byte access of
// r and p) per step when C is even. x is fp32: it never enters the
// recurrence, and each update is formed in fp64 and rounded once.
__global__ __launch_bounds__(kBlock) void k_cg_dir(float* __restrict__ x, const double* __restrict__ r,
                                                   double* __restrict__ p, int64_t nC, int C,
                                                   const CgState* __restrict__ st) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if ((C & 1) == 0) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    typedef float f2 __attribute__((ext_vector_type(2)));
    f2* x2 = (f2*)x;
    d2* p2 = (d2*)p;
    const d2* r2 = (const d2*)r;
    for (int64_t h = t0; h < nC / 2; h += stride) {
      const int c = (int)((2 * h) % C);
      const d2 pv = p2[h], rv = r2[h];
      const f2 xv = x2[h];
      f2 xo;
      d2 po;
      xo[0] = (float)__builtin_fma(st->alpha[c], pv[0], (double)xv[0]);
      xo[1] = (float)__builtin_fma(st->alpha[c + 1], pv[1], (double)xv[1]);
      po[0] = st->active[c] ? __builtin_fma(st->beta[c], pv[0], rv[0]) : pv[0];
      po[1] = st->active[c + 1] ? __builtin_fma(st->beta[c + 1], pv[1], rv[1]) : pv[1];
      x2[h] = xo;
      p2[h] = po;
    }
  } else {
    for (int64_t e = t0; e < nC; e += stride) {
      const int c = (int)(e % C);
      const double pv = p[e];
      x[e] = (float)__builtin_fma(st->alpha[c], pv, (double)x[e]);
      if (st->active[c]) p[e] = __builtin_fma(st->beta[c], pv, r[e]);
    }
  }
}

}  // namespace

int launch_cg_alpha(const double* u, const double* bu, int64_t m, int C, double scale, const CgMvm& cg,
                    hipStream_t s) {
  const int64_t blocks = cg.lat_parts + (cg.ntiles + 15) / 16;
  const int fold = blocks <= kAlphaFoldBlocks ? 1 : 0;
  {
    ProfScope ps(KK_CG_ALPHA, s);
    const size_t lds = fold ? std::max(cg_vec_lds(C), sizeof(double) * kFold * C) : cg_vec_lds(C);
    hipLaunchKernelGGL(k_cg_alpha, dim3((unsigned)blocks), dim3(kBlock), lds, s, u, bu, m, C, scale,
                       cg.lat_parts, (const double*)cg.pp, cg.ntiles, cg.alpha, fold);
    SGP_LAUNCH_CHECK("k_cg_alpha");
  }
  if (!fold) {
    ProfScope ps(KK_CG_SCALAR, s);
    hipLaunchKernelGGL(k_cg_scalar, dim3(1), dim3(kScalarThreads), 0, s, cg.alpha, C);
    SGP_LAUNCH_CHECK("k_cg_scalar");
  }
  return SGP_OK;
}

int launch_cg_dir(const CgDirUpdate& up, int64_t nC, int C, hipStream_t s) {
  ProfScope ps(KK_CG_DIR, s);
  const dim3 grid((unsigned)std::min<int64_t>((nC / 2 + kBlock - 1) / kBlock + 1, 65536));
  hipLaunchKernelGGL(k_cg_dir, grid, dim3(kBlock), 0, s, up.x, up.r, up.p, nC, C, up.st);
  SGP_LAUNCH_CHECK("k_cg_dir");
  return SGP_OK;
}

namespace {

// x back to the caller's order: one thread per (row, four channels). When
// the direction update runs in the splat (p non-null), the last iteration's
// x += alpha p is still due and is applied here, as the update would.
__global__ __launch_bounds__(kBlock) void k_cg_out(const float* __restrict__ xs,
                                                   const uint32_t* __restrict__ perm,
                                                   float* __restrict__ x, int64_t n, int C, int vec,
                                                   const double* __restrict__ p,
                                                   const CgState* __restrict__ st) {
  const int ng = (C + 3) / 4;
  const int64_t total = n * ng;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    const int64_t i = t / ng;
    const int c = (int)(t - i * ng) * 4;
    const float* src = xs + i * C + c;
    float* dst = x + (int64_t)perm[i] * C + c;
    float v[4];
    if (vec) {
      const float4 a = *(const float4*)src;
      v[0] = a.x;
      v[1] = a.y;
      v[2] = a.z;
      v[3] = a.w;
    } else {
      for (int k = 0; k < 4; ++k) v[k] = c + k < C ? src[k] : 0.f;
    }
    if (p) {
      for (int k = 0; k < 4 && c + k < C; ++k)
        v[k] = (float)__builtin_fma(st->alpha[c + k], p[i * C + c + k], (double)v[k]);
    }
    if (vec) {
      *(float4*)dst = make_float4(v[0], v[1], v[2], v[3]);
    } else {
      for (int k = 0; k < 4 && c + k < C; ++k) dst[k] = v[k];
    }
  }
}

// The last solve's idle graph on this thread (a plain thread-local pair, so
// nothing runs at thread or process exit).
thread_local hipGraph_t t_idle_graph = nullptr;
thread_local hipGraphExec_t t_idle_exec = nullptr;

void retire_graphs() {
  if (t_idle_exec) (void)hipGraphExecDestroy(t_idle_exec);
  if (t_idle_graph) (void)hipGraphDestroy(t_idle_graph);
  t_idle_exec = nullptr;
  t_idle_graph = nullptr;
}

void defer_graph(hipGraph_t g, hipGraphExec_t e) {
  retire_graphs();
  t_idle_graph = g;
  t_idle_exec = e;
}

int cg_run(const sgp_lattice* L, const float* b, int C, float noise, float tol, int max_iter,
           float* x, int32_t* iters, float* rel, hipStream_t s) {
  sgp_lattice* Lm = const_cast<sgp_lattice*>(L);
  const int64_t n = L->n, nC = n * C;
  int rc;
  // r, p in fp64, then x in fp32
  if ((rc = dev_reserve(L, Lm->cgvec, (sizeof(double) * 2 + sizeof(float)) * nC, s))) return rc;
  // partial sums: one row per superchunk from the init kernel or per tile
  // from the slice (r.r); one per superchunk of lattice rows and per 16
  // tiles (alpha); one per tile from the splat (p.p); then the scalar
  // state, and the finished-block counter of the last-block folds
  const int64_t iparts = cg_supers(n, kSuperInit);
  const int64_t lparts = cg_supers(L->m, kSuperLat), groups = (L->ntiles + 15) / 16;
  const int64_t rparts = std::max(L->ntiles, iparts);
  auto rows_bytes = [&](int64_t rows) { return ((sizeof(double) * rows * C + 255) / 256) * 256; };
  const size_t rr_bytes = rows_bytes(rparts), al_bytes = rows_bytes(lparts + groups);
  const size_t pp_bytes = rows_bytes(L->ntiles);
  const size_t st_bytes = ((sizeof(CgState) + 255) / 256) * 256;
  const size_t red_bytes = rr_bytes + al_bytes + pp_bytes + st_bytes + 256;
  if ((rc = dev_reserve(L, Lm->cgred, red_bytes, s))) return rc;
  double* r = (double*)Lm->cgvec.ptr;
  double* p = r + nC;
  float* x32 = (float*)(p + nC);
  char* red = (char*)Lm->cgred.ptr;
  double* rr_parts = (double*)red;
  double* al_parts = (double*)(red + rr_bytes);
  double* pp_parts = (double*)(red + rr_bytes + al_bytes);
  CgState* st = (CgState*)(red + rr_bytes + al_bytes + pp_bytes);
  unsigned* counter = (unsigned*)(red + rr_bytes + al_bytes + pp_bytes + st_bytes);

  int32_t* host = (int32_t*)pinned_scratch(sizeof(int32_t) * 3 * kMaxCgCols);
  if (!host) {
    set_error("cg_solve: pinned host scratch unavailable");
    return SGP_ENOMEM;
  }

  const dim3 block(kBlock);
  const dim3 igrid((unsigned)std::min<int64_t>(iparts, 65536));
  const size_t vlds = cg_vec_lds(C);
  const CgHook h_start{rr_parts, iparts, st, counter, (int)SM_START, (double)tol};
  CgMvm cgm;
  cgm.alpha = CgHook{al_parts, lparts + groups, st, counter, (int)SM_ALPHA, (double)tol};
  cgm.lat_parts = lparts;
  cgm.pp = pp_parts;
  cgm.ntiles = L->ntiles;
  cgm.beta = CgHook{rr_parts, L->ntiles, st, counter, (int)SM_BETA, (double)tol};
  cgm.r = r;
  if ((rc = launch_fill_u32(counter, 1, 0u, s))) return rc;
  {
    ProfScope ps(KK_CG_INIT, s);
    hipLaunchKernelGGL(k_cg_init, igrid, block, vlds, s, b, (const uint32_t*)L->perm.ptr, x32, r, p, n, C,
                       L->solve_rows, rr_parts);
    SGP_LAUNCH_CHECK("k_cg_init");
  }
  {
    ProfScope ps(KK_CG_SCALAR, s);
    hipLaunchKernelGGL(k_cg_scalar, dim3(1), dim3(kScalarThreads), 0, s, h_start, C);
    SGP_LAUNCH_CHECK("k_cg_scalar");
  }
  // One iteration: one MVM of p that also yields alpha, r -= alpha A p,
  // convergence and beta (CgMvm); x and p move in the next iteration's
  // splat. Nothing here talks to the host, so a block of iterations can be
  // recorded as a graph.
  // The direction update x += alpha p, p = r + beta p of an iteration runs
  // in the next iteration's splat (CgDirUpdate), or as a pass of its own
  // when that fusion is switched off; both give the same values bit for bit.
  const bool fused = cg_fuse_enabled();
  const CgDirUpdate dirup{p, r, x32, st};
  auto iterate = [&](hipStream_t st_, bool first) -> int {
    int rc_ = mvm_cg(L, p, C, st_, (double)noise, cgm, (fused && !first) ? &dirup : nullptr);
    if (rc_) return rc_;
    if (!fused) {
      const int rc2 = launch_cg_dir(dirup, nC, C, st_);
      if (rc2) return rc2;
    }
    return SGP_OK;
  };
  // Polls read the per-column active flags; each one drains the queue, so
  // none are made when the caller asked for a fixed iteration count.
  auto all_done = [&](bool* done) -> int {
    SGP_HIP(hipMemcpyAsync(host, st->active, sizeof(int32_t) * C, hipMemcpyDeviceToHost, s));
    SGP_HIP(hipStreamSynchronize(s));
    bool any = false;
    for (int c = 0; c < C; ++c) any |= host[c] != 0;
    *done = !any;
    return SGP_OK;
  };
  const bool polling = tol > 0.f;
  const int blk = polling ? 4 : 8;
  // The first iterations run launch by launch: the first MVM sizes the
  // lattice's work buffers (a graph must not allocate). With a tolerance,
  // the first block and one more iteration do, so that a solve converging
  // within them never pays for recording a graph. With a fixed count, the
  // head is what leaves the rest a whole number of blocks (at least one
  // iteration), e.g. 4 + 2 x 8 for 20 iterations.
  int it = 0;
  bool done = false;
  const int eager_head = polling ? (blk + 1 < max_iter ? blk + 1 : max_iter) : (max_iter - 1) % blk + 1;
  for (; it < eager_head && !done; ++it) {
    if ((rc = iterate(s, it == 0))) return rc;
    if (polling && (it + 1) % blk == 0 && it + 1 < max_iter)
      if ((rc = all_done(&done))) return rc;
  }
  if (!done && polling && it < max_iter && it % blk != 0)
    if ((rc = all_done(&done))) return rc;
  // Tearing a graph down costs the host a few hundred microseconds. A
  // solve's graph is kept until the next solve on this thread has put its
  // first iterations on the GPU and is torn down then, so the GPU does not
  // wait for it; if the function returns early, it is torn down at once.
  retire_graphs();
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  struct GraphGuard {
    hipGraph_t* g;
    hipGraphExec_t* e;
    hipStream_t s;
    bool keep = false;
    ~GraphGuard() {
      if (keep) {
        defer_graph(*g, *e);
        return;
      }
      if (*e) {
        (void)hipStreamSynchronize(s);
        (void)hipGraphExecDestroy(*e);
      }
      if (*g) (void)hipGraphDestroy(*g);
    }
  } guard{&graph, &exec, s};
  if (!done && max_iter - it >= 2 * blk && cg_graphs_enabled() && !profiling()) {
    hipStream_t cs = capture_stream();
    if (!cs) {
      set_error("cg_solve: could not create a capture stream");
      return SGP_EHIP;
    }
    SGP_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    int crc = SGP_OK;
    for (int b = 0; b < blk && !crc; ++b) crc = iterate(cs, false);
    hipError_t ce = hipStreamEndCapture(cs, &graph);
    if (crc) return crc;
    SGP_HIP(ce);
    SGP_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    while (!done && max_iter - it >= blk) {
      SGP_HIP(hipGraphLaunch(exec, s));
      it += blk;
      if (polling && it < max_iter)
        if ((rc = all_done(&done))) return rc;
    }
  }
  for (; it < max_iter && !done; ++it) {
    if ((rc = iterate(s, it == 0))) return rc;
    if (polling && (it + 1) % blk == 0 && it + 1 < max_iter)
      if ((rc = all_done(&done))) return rc;
  }
  {
    ProfScope ps(KK_CG_OUT, s);
    const int vec = (C % 4 == 0 && ((uintptr_t)x & 15u) == 0) ? 1 : 0;
    const int64_t work = n * ((C + 3) / 4);
    hipLaunchKernelGGL(k_cg_out, dim3((unsigned)std::min<int64_t>((work + kBlock - 1) / kBlock, 65536)), block, 0, s,
                       (const float*)x32, (const uint32_t*)L->perm.ptr, x, n, C, vec,
                       fused ? (const double*)p : (const double*)nullptr, (const CgState*)st);
    SGP_LAUNCH_CHECK("k_cg_out");
  }
  SGP_HIP(hipMemcpyAsync(host, st->iters, sizeof(int32_t) * C, hipMemcpyDeviceToHost, s));
  SGP_HIP(hipMemcpyAsync(host + kMaxCgCols, st->rel, sizeof(float) * C, hipMemcpyDeviceToHost, s));
  SGP_HIP(hipStreamSynchronize(s));
  guard.keep = true;  // idle now: torn down during the next solve
  mark_use(L, s);
  for (int c = 0; c < C; ++c) {
    if (iters) iters[c] = host[c];
    if (rel) {
      float v;
      memcpy(&v, &host[kMaxCgCols + c], sizeof(float));
      rel[c] = v;
    }
  }
  return SGP_OK;
}

}  // namespace
}  // namespace sgp

using namespace sgp;

extern "C" int cg_solve(const sgp_lattice* L, const float* rhs, int32_t C, float noise, float tol,
                        int32_t max_iter, float* x, int32_t* iters, float* rel_residual,
                        void* stream) {
  if (!L || !rhs || !x) {
    set_error("cg_solve: NULL argument");
    return SGP_EINVAL;
  }
  if (C < 1 || C > kMaxCgCols) {
    set_error("cg_solve: need 1 <= C <= %d (got %d)", kMaxCgCols, (int)C);
    return SGP_EINVAL;
  }
  if (!(noise >= 0.f) || !std::isfinite(noise) || !(tol >= 0.f) || !std::isfinite(tol) || max_iter < 1) {
    set_error("cg_solve: need finite noise >= 0, finite tol >= 0 and max_iter >= 1");
    return SGP_EINVAL;
  }
  const size_t bytes = sizeof(float) * (size_t)L->n * (size_t)C;
  const char* b0 = (const char*)rhs;
  const char* x0 = (const char*)x;
  if (b0 < x0 + bytes && x0 < b0 + bytes) {
    set_error("cg_solve: x overlaps rhs");
    return SGP_EINVAL;
  }
  return cg_run(L, rhs, C, noise, tol, max_iter, x, iters, rel_residual, (hipStream_t)stream);
}
