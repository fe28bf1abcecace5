// The lattice MVM  out = outputscale * W_X K_UU W_X^T V  (Section 4, eq. ski_to_bf):
//   k_splat  U = W^T V: every (point, vertex) adds w * V[point] into its
//            lattice row with a float atomic (Section 3.2, Splat)
//   k_blur   one step of the blur: U'[j] = sum_t stencil[t] U[nbr(j, k, t)],
//            missing neighbours contributing zero (Section 3.2, Blur); in
//            SYMMETRIC order the forward chain (direction step) and the
//            reverse chain (direction d-step) advance in the same launch
//   k_slice  out = scale * W U, gathering the d+1 vertex rows of every point
//            (Section 3.2, Slice); the CG variant also adds noise * p and
//            emits per-block partial sums of p . out per column
//
// Layout: point-side arrays are n x C row-major, lattice values m x C
// row-major, so the G lanes that share one row (G = the power of two >= C,
// at most 64) read and write it contiguously.
#include "sgp_internal.h"

namespace sgp {
namespace {

template <typename TV, typename TU, int G>
__global__ __launch_bounds__(kBlock) void k_splat(const int32_t* __restrict__ idx,
                                                  const float* __restrict__ w,
                                                  const TV* __restrict__ V,
                                                  TU* __restrict__ U, int64_t n, int D, int C) {
  constexpr int R = kBlock / G;
  const int lane = threadIdx.x % G;
  const int64_t stride = (int64_t)gridDim.x * R;
  for (int64_t i = (int64_t)blockIdx.x * R + threadIdx.x / G; i < n; i += stride) {
    const int32_t* ii = idx + i * D;
    const float* wi = w + i * D;
    for (int c = lane; c < C; c += G) {
      const TU v = (TU)V[i * C + c];
      for (int k = 0; k < D; ++k) unsafeAtomicAdd(&U[(int64_t)ii[k] * C + c], (TU)wi[k] * v);
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
  TU st[2 * kMaxOrder + 1];
};

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename TU, int G>
__global__ __launch_bounds__(kBlock) void k_blur(BlurArgs<TU> a) {
  constexpr int R = kBlock / G;
  const int lane = threadIdx.x % G;
  const int64_t rows = a.m * a.chains;
  const int64_t stride = (int64_t)gridDim.x * R;
  const int C = a.C, r = a.r;
  for (int64_t q = (int64_t)blockIdx.x * R + threadIdx.x / G; q < rows; q += stride) {
    const int ch = q >= a.m ? 1 : 0;
    const int64_t j = q - (ch ? a.m : 0);
    const TU* in = a.in[ch];
    const int32_t* nb = a.nbr[ch] + j;
    for (int c = lane; c < C; c += G) {
      TU acc = 0;
      int ti = 0;
      for (int t = -r; t <= r; ++t) {
        TU u;
        if (t == 0) {
          u = in[j * C + c];
        } else {
          const int32_t x = nb[(int64_t)ti * a.m];
          u = x >= 0 ? in[(int64_t)x * C + c] : (TU)0;
          ++ti;
        }
        acc = fma_t(a.st[t + r], u, acc);
      }
      a.out[ch][j * C + c] = acc;
    }
  }
}

template <typename TV, typename TU, int G, bool SYM, bool CG>
__global__ __launch_bounds__(kBlock) void k_slice(const int32_t* __restrict__ idx,
                                                  const float* __restrict__ w,
                                                  const TU* __restrict__ UF,
                                                  const TU* __restrict__ UR,
                                                  TV* __restrict__ out, int64_t n, int D, int C,
                                                  TU scale, TV noise,
                                                  const TV* __restrict__ p,
                                                  double* __restrict__ partials) {
  constexpr int R = kBlock / G;
  const int lane = threadIdx.x % G;
  const int64_t stride = (int64_t)gridDim.x * R;
  double dot = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * R + threadIdx.x / G; i < n; i += stride) {
    const int32_t* ii = idx + i * D;
    const float* wi = w + i * D;
    for (int c = lane; c < C; c += G) {
      TU acc = 0;
      for (int k = 0; k < D; ++k) {
        const int64_t row = (int64_t)ii[k] * C + c;
        TU u = UF[row];
        if (SYM) u += UR[row];
        acc = fma_t((TU)wi[k], u, acc);
      }
      TV o = (TV)(scale * acc);
      if (CG) {
        const TV pv = p[i * C + c];
        o = fma_t(noise, pv, o);
        dot += (double)pv * (double)o;
      }
      out[i * C + c] = o;
    }
  }
  if (CG) {
    __shared__ double sh[kBlock];
    sh[threadIdx.x] = dot;
    __syncthreads();
    if ((int)threadIdx.x < C) {
      double s = 0.0;
      for (int rr = 0; rr < R; ++rr) s += sh[rr * G + threadIdx.x];
      partials[(int64_t)blockIdx.x * C + threadIdx.x] = s;
    }
  }
}

unsigned grid_rows(int64_t rows, int G, int64_t cap) {
  const int64_t R = kBlock / G;
  int64_t b = (rows + R - 1) / R;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

template <typename TV, typename TU, int G>
int launch_splat(const sgp_lattice* L, const TV* V, int C, TU* U, hipStream_t s) {
  ProfScope ps(KK_SPLAT, s);
  hipLaunchKernelGGL((k_splat<TV, TU, G>), dim3(grid_rows(L->n, G, 32768)), dim3(kBlock), 0, s,
                     (const int32_t*)L->idx.ptr, (const float*)L->w.ptr, V, U, L->n, L->d + 1, C);
  SGP_LAUNCH_CHECK("k_splat");
  return SGP_OK;
}

template <typename TU, int G>
int launch_blur(const BlurArgs<TU>& a, hipStream_t s) {
  ProfScope ps(KK_BLUR, s);
  hipLaunchKernelGGL((k_blur<TU, G>), dim3(grid_rows(a.m * a.chains, G, 32768)), dim3(kBlock), 0, s, a);
  SGP_LAUNCH_CHECK("k_blur");
  return SGP_OK;
}

template <typename TV, typename TU, int G, bool SYM, bool CG>
int launch_slice(const sgp_lattice* L, const TU* UF, const TU* UR, TV* out, int C, TU scale,
                 TV noise, const TV* p, double* partials, hipStream_t s) {
  ProfScope ps(KK_SLICE, s);
  const unsigned grid = CG ? (unsigned)kRedBlocks : grid_rows(L->n, G, 32768);
  hipLaunchKernelGGL((k_slice<TV, TU, G, SYM, CG>), dim3(grid), dim3(kBlock), 0, s,
                     (const int32_t*)L->idx.ptr, (const float*)L->w.ptr, UF, UR, out, L->n,
                     L->d + 1, C, scale, noise, p, partials);
  SGP_LAUNCH_CHECK("k_slice");
  return SGP_OK;
}

template <typename TV, typename TU, int G>
int mvm_g(const sgp_lattice* L, const TV* V, int C, TV* out, hipStream_t s, TV noise, const TV* p,
          double* partials) {
  const int d = L->d, T = 2 * L->order;
  const int64_t m = L->m, mC = m * C;
  TU* U0 = (TU*)L->ubuf.ptr;
  TU* B1 = U0 + mC;
  TU* B2 = B1 + mC;
  TU* B3 = B2 + mC;
  int rc;
  if ((rc = launch_fill_u32((uint32_t*)U0, (size_t)mC * sizeof(TU) / 4, 0u, s))) return rc;
  if ((rc = launch_splat<TV, TU, G>(L, V, C, U0, s))) return rc;

  const bool sym = L->blur == SGP_BLUR_SYMMETRIC;
  BlurArgs<TU> a;
  a.m = m;
  a.C = C;
  a.r = L->order;
  a.chains = sym ? 2 : 1;
  for (int t = 0; t < 2 * L->order + 1; ++t) a.st[t] = (TU)L->stencil64[t];
  const int32_t* nbr = (const int32_t*)L->nbr.ptr;
  const TU* cur[2] = {U0, U0};
  for (int step = 0; step <= d; ++step) {
    // chain 0: forward (or the single requested order); chain 1: reverse
    const int k0 = (L->blur == SGP_BLUR_REVERSE) ? d - step : step;
    const int k1 = d - step;
    TU* dst0 = (step % 2 == 0) ? B1 : B2;
    TU* dst1 = (step % 2 == 0) ? B3 : U0;
    a.in[0] = cur[0];
    a.out[0] = dst0;
    a.nbr[0] = nbr + (int64_t)k0 * T * m;
    a.in[1] = cur[1];
    a.out[1] = dst1;
    a.nbr[1] = nbr + (int64_t)k1 * T * m;
    if ((rc = launch_blur<TU, G>(a, s))) return rc;
    cur[0] = dst0;
    cur[1] = dst1;
  }
  const bool cg = partials != nullptr;
  const TU scale = sym ? (TU)(0.5 * (double)L->outputscale) : (TU)L->outputscale;
  if (sym) {
    return cg ? launch_slice<TV, TU, G, true, true>(L, cur[0], cur[1], out, C, scale, noise, p, partials, s)
              : launch_slice<TV, TU, G, true, false>(L, cur[0], cur[1], out, C, scale, (TV)0, nullptr, nullptr, s);
  }
  return cg ? launch_slice<TV, TU, G, false, true>(L, cur[0], nullptr, out, C, scale, noise, p, partials, s)
            : launch_slice<TV, TU, G, false, false>(L, cur[0], nullptr, out, C, scale, (TV)0, nullptr, nullptr, s);
}

template <typename TV, typename TU>
int mvm_dispatch(const sgp_lattice* L, const TV* V, int C, TV* out, hipStream_t s, TV noise,
                 const TV* p, double* partials) {
  int rc = dev_reserve(const_cast<sgp_lattice*>(L)->ubuf, sizeof(TU) * 4 * L->m * C);
  if (rc) return rc;
  switch (lanes_for(C)) {
    case 1: return mvm_g<TV, TU, 1>(L, V, C, out, s, noise, p, partials);
    case 2: return mvm_g<TV, TU, 2>(L, V, C, out, s, noise, p, partials);
    case 4: return mvm_g<TV, TU, 4>(L, V, C, out, s, noise, p, partials);
    case 8: return mvm_g<TV, TU, 8>(L, V, C, out, s, noise, p, partials);
    case 16: return mvm_g<TV, TU, 16>(L, V, C, out, s, noise, p, partials);
    case 32: return mvm_g<TV, TU, 32>(L, V, C, out, s, noise, p, partials);
    default: return mvm_g<TV, TU, 64>(L, V, C, out, s, noise, p, partials);
  }
}

}  // namespace

int mvm_into(const sgp_lattice* L, const float* V, int C, float* out, hipStream_t s) {
  return mvm_dispatch<float, float>(L, V, C, out, s, 0.f, nullptr, nullptr);
}

int mvm_cg(const sgp_lattice* L, const double* p, int C, double* q, hipStream_t s, double noise,
           double* partials) {
  return mvm_dispatch<double, double>(L, p, C, q, s, noise, p, partials);
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
  return mvm_into(L, values, C, out, (hipStream_t)stream);
}
