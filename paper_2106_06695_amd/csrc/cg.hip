// Conjugate gradients on (outputscale*K + noise*I) x = b, one independent
// recurrence per column (Section 2, Krylov methods; Section 5.4 on
// tolerances). All scalars stay on the device: the slice of each MVM emits
// per-block partial sums of p.q, a one-block kernel turns them into alpha,
// the update kernel moves x and r and emits partial sums of r.r, and a
// second one-block kernel decides convergence and beta. The host only polls
// the per-column "active" flags every few iterations.
//
// Precision: the solver's vectors (x, r, p, q), the lattice values inside
// its MVMs and all reductions are fp64; only the barycentric weights stay
// fp32. In fp32 the recursive residual drifts from the true one by about
// eps * cond(A), which at the conditioning of typical GP systems
// (cond ~ 1e3..1e4) is already above a 1e-4 tolerance. The caller's rhs and
// x are fp32. Partial sums are reduced in a fixed order, so a run is
// reproducible given the MVM's own rounding.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "sgp_internal.h"

namespace sgp {
namespace {

struct CgState {
  double rr[kMaxCgCols];
  double bnorm[kMaxCgCols];
  double alpha[kMaxCgCols];
  double beta[kMaxCgCols];
  float rel[kMaxCgCols];
  int32_t active[kMaxCgCols];
  int32_t iters[kMaxCgCols];
};

enum ScalarMode { SM_START = 0, SM_ALPHA = 1, SM_BETA = 2 };

// Vectors live in the lattice's internal point order: b is gathered through
// the permutation here and x scattered back in k_cg_out.
// The vector kernels give one partial sum per column for every chunk of
// kCgChunk rows: 16 groups of 8 rows, each group added in row order, then the
// 16 group sums in order. The order depends on the rows only, not on how
// many columns are solved together, so a column's iterates are the same alone
// or in a batch. A block takes kCpb(C) chunks at a time; thread (chunk,
// group, column) has the column fastest, so the threads of a group read
// whole rows.
constexpr int kCgChunk = 128;
constexpr int kCgGroups = 16;
constexpr int kCgRowsPerGroup = kCgChunk / kCgGroups;
__host__ __device__ inline int64_t cg_chunks(int64_t n) { return (n + kCgChunk - 1) / kCgChunk; }
__host__ __device__ inline int cg_cpb(int C) {
  const int per = kCgGroups * C;
  return per >= kBlock ? 1 : kBlock / per;
}

// In LDS: the group sums of the block's chunks, [chunk][group][column].
__device__ inline void cg_fold(double* sh, int64_t chunk0, int cpb, int64_t nchunks, int C,
                               double* __restrict__ partials) {
  __syncthreads();
  for (int q = threadIdx.x; q < cpb * C; q += blockDim.x) {
    const int ck = q / C, c = q - ck * C;
    if (chunk0 + ck >= nchunks) continue;
    double v = 0.0;
    for (int g = 0; g < kCgGroups; ++g) v += sh[(ck * kCgGroups + g) * C + c];
    partials[(chunk0 + ck) * C + c] = v;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_cg_init(const float* __restrict__ b,
                                                    const uint32_t* __restrict__ perm,
                                                    double* __restrict__ x,
                                                    double* __restrict__ r, double* __restrict__ p,
                                                    int64_t n, int C, int64_t rows,
                                                    double* __restrict__ partials) {
  __shared__ double sh[kCgGroups * kMaxCgCols];
  const int cpb = cg_cpb(C);
  const int64_t nchunks = cg_chunks(n);
  for (int64_t chunk0 = (int64_t)blockIdx.x * cpb; chunk0 < nchunks; chunk0 += (int64_t)gridDim.x * cpb) {
    for (int q = threadIdx.x; q < cpb * kCgGroups * C; q += blockDim.x) {
      const int c = q % C, gq = q / C;  // gq = chunk * groups + group
      const int64_t i0 = (chunk0 + gq / kCgGroups) * kCgChunk + (gq % kCgGroups) * kCgRowsPerGroup;
      double dot = 0.0;
      for (int64_t i = i0; i < i0 + kCgRowsPerGroup && i < n; ++i) {
        const int64_t e = i * C + c;
        const int64_t src = perm[i];
        const double v = (rows > 0 && src >= rows) ? 0.0 : (double)b[src * C + c];
        x[e] = 0.0;
        r[e] = v;
        p[e] = v;
        dot += v * v;
      }
      sh[q] = dot;
    }
    cg_fold(sh, chunk0, cpb, nchunks, C, partials);
  }
}

constexpr int kScalarThreads = 1024;

// Sum the nparts partial rows of each column in a fixed order and apply one
// step of the scalar recurrence. Pair (g, c) sums rows g, g + kFold, ... of
// column c; one thread per column then folds the kFold sums in order. The
// order depends on nparts only, not on the number of columns.
constexpr int kFold = 64;
__global__ __launch_bounds__(kScalarThreads) void k_cg_scalar(const double* __restrict__ partials,
                                                              int64_t nparts, int C,
                                                              CgState* __restrict__ st, int mode,
                                                              double tol) {
  __shared__ double sh[kFold * kMaxCgCols];
  const int tid = threadIdx.x;
  for (int pair = tid; pair < kFold * C; pair += kScalarThreads) {
    const int g = pair / C, c = pair - g * C;
    double s = 0.0;
    int64_t b = g;
    for (; b + 3 * kFold < nparts; b += 4 * kFold) {
      const double a0 = partials[b * C + c];
      const double a1 = partials[(b + kFold) * C + c];
      const double a2 = partials[(b + 2 * kFold) * C + c];
      const double a3 = partials[(b + 3 * kFold) * C + c];
      s += a0;
      s += a1;
      s += a2;
      s += a3;
    }
    for (; b < nparts; b += kFold) s += partials[b * C + c];
    sh[pair] = s;
  }
  __syncthreads();
  if (tid < C) {
    double v = 0.0;
    for (int gg = 0; gg < kFold; ++gg) v += sh[gg * C + tid];
    const int cc = tid;
    if (mode == SM_START) {
      st->rr[cc] = v;
      st->bnorm[cc] = sqrt(v);
      st->active[cc] = v > 0.0 ? 1 : 0;
      st->iters[cc] = 0;
      st->rel[cc] = v > 0.0 ? 1.f : 0.f;
      st->alpha[cc] = 0.0;
      st->beta[cc] = 0.0;
    } else if (mode == SM_ALPHA) {
      if (st->active[cc] && v > 0.0) {
        st->alpha[cc] = st->rr[cc] / v;
      } else {
        st->alpha[cc] = 0.0;
        st->active[cc] = 0;  // converged, or breakdown (p.Ap <= 0)
      }
    } else {
      if (st->active[cc]) {
        st->iters[cc] += 1;
        const double rel = sqrt(v) / st->bnorm[cc];
        st->rel[cc] = (float)rel;
        if (rel <= tol) {
          st->active[cc] = 0;
          st->beta[cc] = 0.0;
        } else {
          st->beta[cc] = v / st->rr[cc];
          st->rr[cc] = v;
        }
      } else {
        st->beta[cc] = 0.0;
      }
    }
  }
}

// r -= alpha q, and the chunk partial sums of r.r (x moves in k_cg_dir,
// which reads p anyway).
__global__ __launch_bounds__(kBlock) void k_cg_update(double* __restrict__ r,
                                                      const double* __restrict__ q_, int64_t n, int C,
                                                      const CgState* __restrict__ st,
                                                      double* __restrict__ partials) {
  __shared__ double sh[kCgGroups * kMaxCgCols];
  const int cpb = cg_cpb(C);
  const int64_t nchunks = cg_chunks(n);
  for (int64_t chunk0 = (int64_t)blockIdx.x * cpb; chunk0 < nchunks; chunk0 += (int64_t)gridDim.x * cpb) {
    for (int q = threadIdx.x; q < cpb * kCgGroups * C; q += blockDim.x) {
      const int c = q % C, gq = q / C;
      const int64_t i0 = (chunk0 + gq / kCgGroups) * kCgChunk + (gq % kCgGroups) * kCgRowsPerGroup;
      const double a = st->alpha[c];
      double dot = 0.0;
#pragma unroll
      for (int k = 0; k < kCgRowsPerGroup; ++k) {
        const int64_t i = i0 + k;
        if (i < n) {
          const int64_t e = i * C + c;
          const double rv = __builtin_fma(-a, q_[e], r[e]);
          r[e] = rv;
          dot += rv * rv;
        }
      }
      sh[q] = dot;
    }
    cg_fold(sh, chunk0, cpb, nchunks, C, partials);
  }
}

// x += alpha p with this iteration's alpha (zero for a column that was
// already converged), then p = r + beta p for the columns still active.
// Element-wise over the n x C arrays, two elements (one 16-byte access) per
// step when C is even.
__global__ __launch_bounds__(kBlock) void k_cg_dir(double* __restrict__ x, const double* __restrict__ r,
                                                   double* __restrict__ p, int64_t nC, int C,
                                                   const CgState* __restrict__ st) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if ((C & 1) == 0) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    d2* x2 = (d2*)x;
    d2* p2 = (d2*)p;
    const d2* r2 = (const d2*)r;
    for (int64_t h = t0; h < nC / 2; h += stride) {
      const int c = (int)((2 * h) % C);
      const d2 pv = p2[h], xv = x2[h], rv = r2[h];
      d2 xo, po;
      xo[0] = __builtin_fma(st->alpha[c], pv[0], xv[0]);
      xo[1] = __builtin_fma(st->alpha[c + 1], pv[1], xv[1]);
      po[0] = st->active[c] ? __builtin_fma(st->beta[c], pv[0], rv[0]) : pv[0];
      po[1] = st->active[c + 1] ? __builtin_fma(st->beta[c + 1], pv[1], rv[1]) : pv[1];
      x2[h] = xo;
      p2[h] = po;
    }
  } else {
    for (int64_t e = t0; e < nC; e += stride) {
      const int c = (int)(e % C);
      const double pv = p[e];
      x[e] = __builtin_fma(st->alpha[c], pv, x[e]);
      if (st->active[c]) p[e] = __builtin_fma(st->beta[c], pv, r[e]);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_cg_out(const double* __restrict__ x64,
                                                   const uint32_t* __restrict__ perm,
                                                   float* __restrict__ x, int64_t count, int C) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += stride) {
    const int64_t i = e / C;
    const int c = (int)(e - i * C);
    x[(int64_t)perm[i] * C + c] = (float)x64[e];
  }
}

template <int G>
int cg_g(const sgp_lattice* L, const float* b, int C, float noise, float tol, int max_iter,
         float* x, int32_t* iters, float* rel, hipStream_t s) {
  sgp_lattice* Lm = const_cast<sgp_lattice*>(L);
  const int64_t n = L->n, nC = n * C;
  int rc;
  if ((rc = dev_reserve(L, Lm->cgvec, sizeof(double) * 4 * nC, s))) return rc;
  // partial sums: one row per chunk from the vector kernels, one row per tile from the slice
  const int64_t vparts = cg_chunks(n);
  const int64_t nparts = L->ntiles > vparts ? L->ntiles : vparts;
  const size_t red_bytes = sizeof(double) * nparts * C + sizeof(CgState) + 256;
  if ((rc = dev_reserve(L, Lm->cgred, red_bytes, s))) return rc;
  double* x64 = (double*)Lm->cgvec.ptr;
  double* r = x64 + nC;
  double* p = r + nC;
  double* q = p + nC;
  double* partials = (double*)Lm->cgred.ptr;
  CgState* st = (CgState*)((char*)Lm->cgred.ptr + ((sizeof(double) * nparts * C + 255) / 256) * 256);

  int32_t* host = (int32_t*)pinned_scratch(sizeof(int32_t) * 3 * kMaxCgCols);
  if (!host) {
    set_error("cg_solve: pinned host scratch unavailable");
    return SGP_ENOMEM;
  }

  const dim3 block(kBlock);
  const dim3 vgrid((unsigned)std::min<int64_t>((vparts + cg_cpb(C) - 1) / cg_cpb(C), 65536));
  const dim3 grid(kRedBlocks);
  const dim3 dgrid((unsigned)std::min<int64_t>((nC / 2 + kBlock - 1) / kBlock + 1, 65536));
  {
    ProfScope ps(KK_CG_INIT, s);
    hipLaunchKernelGGL(k_cg_init, vgrid, block, 0, s, b, (const uint32_t*)L->perm.ptr, x64, r, p, n, C,
                       L->solve_rows, partials);
    SGP_LAUNCH_CHECK("k_cg_init");
  }
  {
    ProfScope ps(KK_CG_SCALAR, s);
    hipLaunchKernelGGL(k_cg_scalar, dim3(1), dim3(kScalarThreads), 0, s, partials, vparts, C, st,
                       (int)SM_START, (double)tol);
    SGP_LAUNCH_CHECK("k_cg_scalar");
  }
  // One iteration: q = A p (with the p.q partials from the slice), alpha,
  // x and r, convergence and beta, p. Nothing here talks to the host, so a
  // block of iterations can be recorded as a graph.
  auto iterate = [&](hipStream_t st_) -> int {
    int rc_ = mvm_cg(L, p, C, q, st_, (double)noise, partials);
    if (rc_) return rc_;
    {
      ProfScope ps(KK_CG_SCALAR, st_);
      hipLaunchKernelGGL(k_cg_scalar, dim3(1), dim3(kScalarThreads), 0, st_, partials, L->ntiles, C, st,
                         (int)SM_ALPHA, (double)tol);
      SGP_LAUNCH_CHECK("k_cg_scalar");
    }
    {
      ProfScope ps(KK_CG_UPDATE, st_);
      hipLaunchKernelGGL(k_cg_update, vgrid, block, 0, st_, r, q, n, C, st, partials);
      SGP_LAUNCH_CHECK("k_cg_update");
    }
    {
      ProfScope ps(KK_CG_SCALAR, st_);
      hipLaunchKernelGGL(k_cg_scalar, dim3(1), dim3(kScalarThreads), 0, st_, partials, vparts, C,
                         st, (int)SM_BETA, (double)tol);
      SGP_LAUNCH_CHECK("k_cg_scalar");
    }
    {
      ProfScope ps(KK_CG_DIR, st_);
      hipLaunchKernelGGL(k_cg_dir, dgrid, block, 0, st_, x64, r, p, nC, C, st);
      SGP_LAUNCH_CHECK("k_cg_dir");
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
  // The first block and one more iteration run launch by launch: the first
  // MVM sizes the lattice's work buffers (a graph must not allocate), and a
  // solve that converges within them never pays for recording a graph.
  int it = 0;
  bool done = false;
  const int eager_head = blk + 1 < max_iter ? blk + 1 : max_iter;
  for (; it < eager_head && !done; ++it) {
    if ((rc = iterate(s))) return rc;
    if (polling && (it + 1) % blk == 0 && it + 1 < max_iter)
      if ((rc = all_done(&done))) return rc;
  }
  if (!done && polling && it < max_iter && it % blk != 0)
    if ((rc = all_done(&done))) return rc;
  if (!done && max_iter - it >= 2 * blk && cg_graphs_enabled() && !profiling()) {
    hipStream_t cs = capture_stream();
    if (!cs) {
      set_error("cg_solve: could not create a capture stream");
      return SGP_EHIP;
    }
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    struct GraphGuard {
      hipGraph_t* g;
      hipGraphExec_t* e;
      hipStream_t s;
      ~GraphGuard() {
        if (*e) {
          (void)hipStreamSynchronize(s);
          (void)hipGraphExecDestroy(*e);
        }
        if (*g) (void)hipGraphDestroy(*g);
      }
    } guard{&graph, &exec, s};
    SGP_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    int crc = SGP_OK;
    for (int b = 0; b < blk && !crc; ++b) crc = iterate(cs);
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
    if ((rc = iterate(s))) return rc;
    if (polling && (it + 1) % blk == 0 && it + 1 < max_iter)
      if ((rc = all_done(&done))) return rc;
  }
  {
    ProfScope ps(KK_CG_OUT, s);
    hipLaunchKernelGGL(k_cg_out, dim3(kRedBlocks), block, 0, s, x64, (const uint32_t*)L->perm.ptr, x, nC, C);
    SGP_LAUNCH_CHECK("k_cg_out");
  }
  SGP_HIP(hipMemcpyAsync(host, st->iters, sizeof(int32_t) * C, hipMemcpyDeviceToHost, s));
  SGP_HIP(hipMemcpyAsync(host + kMaxCgCols, st->rel, sizeof(float) * C, hipMemcpyDeviceToHost, s));
  SGP_HIP(hipStreamSynchronize(s));
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
  hipStream_t s = (hipStream_t)stream;
  switch (lanes_for(C)) {
    case 1: return cg_g<1>(L, rhs, C, noise, tol, max_iter, x, iters, rel_residual, s);
    case 2: return cg_g<2>(L, rhs, C, noise, tol, max_iter, x, iters, rel_residual, s);
    case 4: return cg_g<4>(L, rhs, C, noise, tol, max_iter, x, iters, rel_residual, s);
    case 8: return cg_g<8>(L, rhs, C, noise, tol, max_iter, x, iters, rel_residual, s);
    case 16: return cg_g<16>(L, rhs, C, noise, tol, max_iter, x, iters, rel_residual, s);
    case 32: return cg_g<32>(L, rhs, C, noise, tol, max_iter, x, iters, rel_residual, s);
    default: return cg_g<64>(L, rhs, C, noise, tol, max_iter, x, iters, rel_residual, s);
  }
}
