// Scalar steps of the conjugate-gradient recurrence (Section 2, Krylov
// methods): fold per-chunk partial sums in a fixed order and apply one step.
// The solver's one-block scalar kernel runs it after a vector kernel; the
// slice's CG variant runs it in its last block to finish, which saves a
// launch where the kernel has few (persistent) blocks.
#ifndef SGP_CG_STEP_H
#define SGP_CG_STEP_H
#include "sgp_internal.h"

namespace sgp {

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

// The previous iteration's direction update, applied by the next MVM's
// splat as it stages the direction (the splat reads p anyway): x += alpha p
// with that iteration's alpha, then p = r + beta p for the columns still
// active, p updated in place. p == nullptr: no update (the first iteration).
struct CgDirUpdate {
  double* p;
  const double* r;
  float* x;
  const CgState* st;
};

// What a partial-sum kernel needs to finish the step itself.
struct CgHook {
  double* partials;   // nparts x C
  int64_t nparts;
  CgState* st;
  unsigned* counter;  // blocks finished; 0 between launches
  int mode;
  double tol;
};

// What the MVM of a CG iteration does besides A p. Its alpha needs p.Ap,
// which equals scale * u.(B u) + noise * p.p for the splatted u = W^T p and
// the blurred B u (the quadratic form of W B W^T taken on the lattice), so
// it is known before the slice, and the slice moves r itself.
//   pp:    row t gets noise * p.p of tile t (from the splat).
//   alpha: rows [0, lat_parts) of its partials get scale * u.Bu of a
//          block of lattice rows, the rows after them the sums of 16
//          consecutive pp rows; a one-block launch folds them into alpha.
//   beta:  row t of its partials gets the new r.r of tile t (from the
//          slice, which updates r in place); its last block folds beta.
struct CgMvm {
  CgHook alpha;
  int64_t lat_parts;
  double* pp;
  int64_t ntiles;
  CgHook beta;
  double* r;
};

constexpr int kFold = 64;  // fixed fold width: the order depends on nparts only

// Sum the nparts partial rows of each column in a fixed order and apply one
// step of the scalar recurrence. Pair (g, c) sums rows g, g + kFold, ... of
// column c; one thread per column folds the kFold sums in order. Called by
// every thread of one block; sh holds kFold * C doubles.
__device__ inline void cg_scalar_block(const double* partials, int64_t nparts, int C, CgState* st,
                                       int mode, double tol, double* sh) {
  const int tid = threadIdx.x;
  for (int pair = tid; pair < kFold * C; pair += blockDim.x) {
    const int g = pair / C, c = pair - g * C;
    constexpr int U = 16;  // loads in flight, then added in row order
    double s = 0.0;
    int64_t b = g;
    for (; b + (U - 1) * kFold < nparts; b += U * kFold) {
      double a[U];
#pragma unroll
      for (int u = 0; u < U; ++u) a[u] = partials[(b + u * kFold) * C + c];
#pragma unroll
      for (int u = 0; u < U; ++u) s += a[u];
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

// Called by every thread of every block at the end of a partial-sum kernel
// (after the block's partials are written): the last block to arrive folds
// them. One thread per block fences and counts: the barrier orders the
// block's partial stores before its release fence, and the last block's
// acquire fence before the barrier that precedes its fold. (A device-scope
// fence writes back or invalidates the L2 of its XCD, so one per block, not
// one per wave.) The last block resets the counter for the next launch.
__device__ inline void cg_finish(const CgHook& h, int C, double* sh) {
  __shared__ int last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned done = atomicAdd(h.counter, 1u);
    last = done == gridDim.x - 1 ? 1 : 0;
    if (last) __threadfence();
  }
  __syncthreads();
  if (!last) return;
  cg_scalar_block(h.partials, h.nparts, C, h.st, h.mode, h.tol, sh);
  if (threadIdx.x == 0) *h.counter = 0u;
}

}  // namespace sgp
#endif  // SGP_CG_STEP_H
